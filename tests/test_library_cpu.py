"""Host-side tests of the C-ABI library (no GPU needed): exported symbols,
the opcode enum against the binding, load-time validation, planning, and
hiprtc compilation into the code cache."""

import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import paper_2408_09662_amd as xg
from paper_2408_09662_amd import _abi
from workloads import configs
from workloads.pendulum import pendulum
from workloads.tracer import Program as WProg, worked_example

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xg_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (xg_[a-z_]+)\b", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        assert f in _abi._SIGS, f"binding lacks a signature for {f}"


def test_opcode_enum_matches_binding():
    text = open(HEADER).read()
    body = text[text.index("XG_OP_INPUT = 0"):text.index("XG_OP_COUNT")]
    names = re.findall(r"XG_OP_([A-Z0-9]+)", body)
    assert names == _abi.OPS


def test_options_struct_matches_header():
    text = open(HEADER).read()
    body = text[text.index("typedef struct {\n  int32_t block;"):text.index("} xg_options;")]
    fields = re.findall(r"int32_t (\w+);", body)
    assert fields == _abi.OPTION_FIELDS


def _load(prog, **opts):
    return xg.Program(prog, **opts)


@pytest.mark.parametrize("instrs,nnz_out,msg", [
    ([("ADD", 0, 1, 1), ("OUTPUT", 0, 0, 0)], [1], "read before write at instruction 0"),
    ([("INPUT", 0, 0, 0), ("OUTPUT", 0, 0, 0)], [2], "output 0[1] never written"),
    ([("INPUT", 0, 0, 3), ("OUTPUT", 0, 0, 0)], [1], "input index out of range at instruction 0"),
    ([("INPUT", 5, 0, 0), ("OUTPUT", 0, 5, 0)], [1], "slot out of range"),
    ([("CONST", 0, 4, -1), ("OUTPUT", 0, 0, 0)], [1], "const index out of range"),
    ([("INPUT", 0, 0, 0), ("OUTPUT", 2, 0, 0)], [1], "output index out of range at instruction 1"),
])
def test_validation_errors(instrs, nnz_out, msg):
    p = WProg("bad", "f64", 2, [1], nnz_out, [1.5], instrs)
    with pytest.raises(xg.XgError) as e:
        _load(p)
    assert "XG_EINVAL" in str(e.value) and msg in str(e.value)


def test_unknown_opcode_rejected():
    d = dict(name="u", dtype="f64", n_work=1, nnz_in=[1], nnz_out=[1], consts=np.zeros(0),
             instr=np.array([[0, 0, 0, 0], [99, 0, 0, 0], [1, 0, 0, 0]], dtype=np.int32))
    with pytest.raises(xg.XgError, match="unknown op 99 at instruction 1"):
        xg.Program(d)


def test_bad_options_rejected():
    with pytest.raises(xg.XgError, match="block"):
        _load(worked_example(), block=96)
    with pytest.raises(xg.XgError, match="ipt"):
        _load(worked_example(), ipt=3)
    with pytest.raises(xg.XgError, match="unknown options"):
        _load(worked_example(), warp=32)


def test_shared_divisors_become_reciprocals():
    """a/b and c/b compile to one reciprocal and two multiplications (not
    in strict mode); b/a keeps its division."""
    from workloads.tracer import Graph
    g = Graph("recip", "f64")
    a, b, c = g.input(3)
    prog = g.program([[a / b, c / b, b / a]])
    p = _load(prog)
    assert p.info(0)["n_ops"] == 4  # 1/b, a*(1/b), c*(1/b), b/a
    assert _load(prog, strict=1).info(0)["n_ops"] == 3


def test_slot_reuse_becomes_ssa():
    # the worked example reuses slot 1 twice: 3 SSA operations remain
    info = _load(worked_example()).info(0)
    assert info["n_ops"] == 3 and info["n_nodes"] == 4 and info["n_chunks"] == 1


def test_dead_code_and_common_subexpressions_removed():
    ins = [("INPUT", 0, 0, 0), ("SIN", 1, 0, -1), ("SIN", 2, 0, -1), ("ADD", 3, 1, 2),
           ("COS", 1, 0, -1),  # dead: overwritten below without being read
           ("MUL", 1, 3, 3), ("OUTPUT", 0, 1, 0)]
    info = _load(WProg("d", "f64", 4, [1], [1], [], ins)).info(0)
    assert info["n_ops"] == 3  # sin (merged), add, mul


def test_plan_facts_pendulum_and_workspace():
    p = xg.Program(configs.program_path("pend7"))
    i0 = p.info(0)
    # 140 divisions by 28 distinct divisors become 28 reciprocals and 112
    # multiplications (28 more operations); strict mode keeps them
    assert i0["n_ops"] == 15354 + 28 and i0["n_chunks"] == 1
    assert xg.Program(configs.program_path("pend7"), strict=1).info(0)["n_ops"] == 15354
    assert p.workspace_bytes(16384, 0) == i0["n_ws_slots"] * 16384 * 8
    p2 = xg.Program(configs.program_path("pend7"), chunk_ops=4000)
    i2 = p2.info(0)
    assert i2["n_chunks"] >= 4 and i2["n_ws_slots"] > 0
    assert p2.workspace_bytes(1000, 0) == i2["n_ws_slots"] * 1024 * 8  # pitch rounded to 64
    a = p.info(2)
    assert a["n_ops"] > 2 * i0["n_ops"]


def test_precompile_without_gpu(tmp_path, monkeypatch):
    monkeypatch.setenv("XG_CACHE_DIR", str(tmp_path))
    monkeypatch.setenv("XG_NO_CACHE", "1")
    p = _load(worked_example())
    p.precompile(0)
    p.precompile(2)
    files = sorted(os.listdir(tmp_path))
    assert len(files) == 2 and all(f.startswith("xg-") and f.endswith(".co") for f in files)
    data = open(tmp_path / files[0], "rb").read()
    assert data[:4] == b"\x7fELF"
    monkeypatch.delenv("XG_NO_CACHE")
    q = _load(worked_example())
    q.precompile(0)
    assert q.info(0)["cache_hits"] == 1


def test_autotune_candidates_precompile_without_gpu(tmp_path, monkeypatch):
    """Every plan the autotuner would time compiles; larger instance counts
    add the occupancy-fitting LDS budget and the 4-wave workgroup."""
    monkeypatch.setenv("XG_CACHE_DIR", str(tmp_path))
    p = _load(worked_example())
    xg.autotune_precompile(p, 1000)
    small = len(os.listdir(tmp_path))
    xg.autotune_precompile(p, 1 << 18)
    large = len(os.listdir(tmp_path))
    assert small >= 1 and large > small  # a tiny program plans alike at every budget
    with pytest.raises(xg.XgError):
        xg.autotune_precompile(p, 0)


def test_adjoint_options_are_separate(tmp_path, monkeypatch):
    """The adjoint modes carry their own options: their autotune candidates
    compile without a GPU, and options of one mode leave the other's plan
    alone."""
    monkeypatch.setenv("XG_CACHE_DIR", str(tmp_path))
    p = xg.Program(configs.program_path("rdag200"))
    assert p.effective_options(0) == p.effective_options(1) == p.effective_options(2)
    xg.autotune_precompile(p, 1 << 16, 2)
    xg.autotune_precompile(p, 1 << 16, 1)
    assert len(os.listdir(tmp_path)) > 2
    with pytest.raises(xg.XgError):
        xg.autotune_precompile(p, 1000, 3)
    with pytest.raises(xg.XgError):
        p.effective_options(3)


def test_generated_source_has_no_scratch_and_fits_registers(tmp_path, monkeypatch):
    """The register plan keeps the generated kernels spill-free; the
    library reads the register count from the kernel descriptor (as
    llvm-readelf reports it), which is what it checks against the launch's
    workgroup size before loading a kernel."""
    monkeypatch.setenv("XG_CACHE_DIR", str(tmp_path))
    p = xg.Program(configs.program_path("rdag200"))
    p.precompile(0)
    co = os.path.join(tmp_path, os.listdir(tmp_path)[0])
    notes = subprocess.run(["/opt/rocm/llvm/bin/llvm-readelf", "--notes", co], capture_output=True,
                           text=True).stdout
    assert ".private_segment_fixed_size: 0" in notes
    vg = [int(v) for v in re.findall(r"\.vgpr_count:\s+(\d+)", notes)]
    assert vg and max(vg) <= 256
    assert p.info(0)["vgprs"] == -(-max(vg) // 8) * 8  # allocated in granules of 8
    q = xg.Program(configs.program_path("pend7"), reg_budget=224, lds_slots=319, prefetch=24)
    q.precompile(0)
    co = [f for f in os.listdir(tmp_path) if os.path.join(tmp_path, f) != co]
    notes = subprocess.run(["/opt/rocm/llvm/bin/llvm-readelf", "--notes", os.path.join(tmp_path, co[0])],
                           capture_output=True, text=True).stdout
    assert q.info(0)["vgprs"] == -(-int(re.findall(r"\.vgpr_count:\s+(\d+)", notes)[0]) // 8) * 8 > 256


def test_precision_tags_validated_and_planned():
    from workloads.tracer import Graph, sin
    g = Graph("m", "f64")
    x = g.input(2)
    with g.precision("f32"):
        y = sin(x[0]) * x[1]
    prog = g.program([[y + x[0]]])
    p = xg.Program(prog)
    assert p.info(0)["n_ops"] == 3
    # the same instructions without tags are different SSA values (no merging across precisions)
    d = xg.load_program_file  # noqa: F841
    bad = WProg("b", "f32", 2, [1], [1], [], [("INPUT", 0, 0, 0), ("SIN", 1, 0, -1), ("OUTPUT", 0, 1, 0)])
    dd = dict(name="b", dtype="f32", n_work=2, nnz_in=[1], nnz_out=[1], consts=np.zeros(0),
              instr=np.array([[0, 0, 0, 0], [13, 1, 0, -1], [1, 0, 1, 0]], dtype=np.int32),
              prec=np.array([0, 64, 0], dtype=np.int8))
    with pytest.raises(xg.XgError, match="precision tag"):
        xg.Program(dd)
    del bad


def test_mixed_program_source_is_typed(tmp_path, monkeypatch):
    from workloads.tracer import Graph, sin
    monkeypatch.setenv("XG_DUMP_DIR", str(tmp_path))
    monkeypatch.setenv("XG_CACHE_DIR", str(tmp_path))
    g = Graph("m", "f64")
    x = g.input(2)
    with g.precision("f32"):
        y = sin(x[0]) * x[1]
    p = xg.Program(g.program([[y + x[0]]]))
    p.precompile(0)
    src = [open(tmp_path / f).read() for f in os.listdir(tmp_path) if f.endswith(".hip")][0]
    assert "const float" in src and "xg_SINf(" in src and "(float)" in src and "(T)" in src


def test_cooperative_tile_plans_and_options():
    """waves > 1: one kernel per evaluation; option validation; the
    planner's own invariant check runs for every program (an error would
    surface here as XgError)."""
    for key in ("rdag200", "pend7"):
        for w in (2, 4, 8, 16):
            p = xg.Program(configs.program_path(key), waves=w)
            i = p.info(0)
            assert i["n_chunks"] == 1 and i["n_ws_slots"] > 0
            assert p.effective_options()["waves"] == w
    with pytest.raises(xg.XgError):
        xg.Program(configs.program_path("rdag200"), waves=3).info(0)
    with pytest.raises(xg.XgError):
        xg.Program(configs.program_path("rdag200"), waves=4, block=128).info(0)


def _code_sections(path):
    """Hex dump of a code object's machine code and kernel descriptors."""
    return subprocess.run(["/opt/rocm/llvm/bin/llvm-readelf", "-x", ".text", "-x", ".rodata", str(path)],
                          capture_output=True, text=True, check=True).stdout.split("\n", 1)[1]


def test_parallel_compile_matches_serial(tmp_path, monkeypatch):
    """The chunks of a large program compile in helper processes, several at
    once; one helper at a time gives the same machine code and kernel
    descriptors, byte for byte (the code objects differ only in the
    compilation-unit id symbol hiprtc draws per compilation)."""
    assert os.access(os.path.join(os.path.dirname(_abi.LIB_PATH), "xg-rtc"), os.X_OK)
    dirs = {}
    for procs in ("1", "4"):
        d = tmp_path / procs
        d.mkdir()
        monkeypatch.setenv("XG_CACHE_DIR", str(d))
        monkeypatch.setenv("XG_COMPILE_PROCS", procs)
        p = xg.Program(configs.program_path("pend7"), chunk_ops=4000)
        p.precompile(0)
        assert p.info(0)["n_chunks"] >= 4 and p.info(0)["cache_hits"] == 0
        dirs[procs] = {f: _code_sections(d / f) for f in os.listdir(d)}
    assert dirs["1"] and dirs["1"] == dirs["4"]
    assert all(f.startswith("xg-") and f.endswith(".co") for f in dirs["4"])  # no helper files left


def test_one_hip_runtime_per_process():
    """The binding loads libxg.so after torch, so both use torch's HIP
    runtime (torch bundles its own copy of the ROCm libraries)."""
    code = ("import paper_2408_09662_amd as xg; xg.lib(); "
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}; "
            "print(len(libs))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True)
    assert out.stdout.strip() == "1"


def test_batch_autotune_workspace_covers_every_candidate():
    """The workspace the batch autotuner asks for covers its 64-lane
    candidate (one lane per instance) and the cooperative ones, which keep
    more values in the workspace."""
    import ctypes
    progs = [xg.Program(configs.program_path(k)) for k in ("rdag1e4", "rdag200", "mpc")]
    ns = [700, 1500, 600]
    arr = (ctypes.c_void_p * 3)(*[p._h.value for p in progs])
    na = (ctypes.c_int64 * 3)(*ns)
    b = ctypes.c_size_t()
    _abi.check(_abi.lib().xg_batch_autotune_workspace_bytes(arr, 3, na, ctypes.byref(b)))
    plain = sum(p.workspace_bytes(n, 0) for p, n in zip(progs, ns))
    wide = xg.Program(configs.program_path("rdag1e4"), waves=8).workspace_bytes(700, 0)
    assert b.value >= plain and b.value >= wide
    with pytest.raises(xg.XgError):
        _abi.check(_abi.lib().xg_batch_autotune_workspace_bytes(arr, 0, na, ctypes.byref(b)))


def test_contraction_is_granted_by_the_source_not_the_compiler(tmp_path, monkeypatch):
    """Outside strict mode a generated source starts with the FMA-contraction
    pragma and is compiled with -ffp-contract=on (a global 'fast' setting
    would also fuse inside the device library's functions); strict mode has
    neither."""
    from workloads.tracer import Graph
    monkeypatch.setenv("XG_DUMP_DIR", str(tmp_path))
    monkeypatch.setenv("XG_CACHE_DIR", str(tmp_path))
    g = Graph("c", "f64")
    a, b, c = g.input(3)
    prog = g.program([[a * b + c]])
    for strict in (0, 1):
        before = set(os.listdir(tmp_path))
        xg.Program(prog, strict=strict).precompile(0)
        src = [f for f in os.listdir(tmp_path) if f.endswith(".hip") and f not in before]
        text = open(tmp_path / src[0]).read()
        assert ("#pragma clang fp contract(fast)" in text) == (strict == 0)



# ------------------------------------------------- code-object host checks

def _checker(tmp_path):
    """Build the test driver of the library's code-object checks."""
    exe = tmp_path / "codeobject_check"
    src = os.path.join(ROOT, "tests", "native", "codeobject_check.cpp")
    libdir = os.path.dirname(_abi.LIB_PATH)
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"), "-I",
                    os.path.join(libdir, "csrc"), src, "-o", str(exe), "-L", libdir, "-l:libxg.so",
                    f"-Wl,-rpath,{libdir}"], check=True)
    return exe


def _check(exe, co, kernel, block, explicit):
    out = subprocess.run([str(exe), str(co), kernel, str(block), str(explicit)], capture_output=True,
                         text=True, check=True).stdout.split()
    regs, lds, scratch, kernarg, hidden, fits, args = (int(v) for v in out)
    return dict(regs=regs, lds=lds, scratch=scratch, kernarg=kernarg, hidden=hidden, fits=fits, args=args)


def test_cooperative_kernel_argument_layout_checked_on_host(tmp_path, monkeypatch):
    """The cooperative-tile kernel's device functions read the arguments as
    one block just before the implicit arguments; the host check reads the
    implicit arguments' offset from the code object's metadata note."""
    cache = tmp_path / "cache"
    cache.mkdir()
    monkeypatch.setenv("XG_CACHE_DIR", str(cache))
    p = xg.Program(configs.program_path("rdag200"), waves=4)
    p.precompile(0)  # runs the host checks too
    cos = sorted(cache.glob("xg-*.co"))
    assert len(cos) == 1
    exe = _checker(tmp_path)
    explicit = 8 * (2 + 2 * (len(p.nnz_in) + len(p.nnz_out)))  # n, (ptr, ld) per argument, ws
    r = _check(exe, cos[0], "xg_m0_c0", 256, explicit)
    assert r["hidden"] == explicit and r["args"] == 1 and r["fits"] == 1
    assert r["kernarg"] > explicit  # the implicit arguments follow
    assert 0 < r["regs"] <= 512 and r["lds"] <= 160 * 1024 and r["scratch"] == 0
    # a block of another size is refused
    assert _check(exe, cos[0], "xg_m0_c0", 256, explicit - 8)["args"] == 0
    assert _check(exe, cos[0], "xg_m0_c0", 256, explicit + 8)["args"] == 0


def test_batch_kernel_argument_layout_and_resources_checked_on_host(tmp_path, monkeypatch):
    cache = tmp_path / "cache"
    cache.mkdir()
    monkeypatch.setenv("XG_CACHE_DIR", str(cache))
    progs = [xg.Program(configs.program_path("rdag200")), xg.Program(worked_example())]
    xg.Batch(progs)  # compiles and checks on the host
    exe = _checker(tmp_path)
    # BArgs: counter, total, cum[K + 1], then per program n, ws and (ptr, ld) per argument
    explicit = 8 + 8 + 8 * (len(progs) + 1) + sum(16 + 16 * (len(p.nnz_in) + len(p.nnz_out)) for p in progs)
    found = [co for co in cache.glob("xg-*.co") if b"xg_batch" in co.read_bytes()]
    assert len(found) == 1
    r = _check(exe, found[0], "xg_batch", 64, explicit)
    assert r["hidden"] == explicit and r["args"] == 1 and r["fits"] == 1
    assert _check(exe, found[0], "xg_batch", 64, explicit + 16)["args"] == 0
    # registers: a 64-lane workgroup fits; the same kernel refused if its
    # waves could not all be resident (a workgroup of 64 x 4 x k waves needs
    # k x regs per SIMD)
    if r["regs"] > 128:
        assert _check(exe, found[0], "xg_batch", 1024, -1)["fits"] == 0


def test_program_info_reports_kernel_resources(tmp_path, monkeypatch):
    monkeypatch.setenv("XG_CACHE_DIR", str(tmp_path))
    p = xg.Program(configs.program_path("pend7"))
    p.precompile(0)
    inf = p.info(0)
    assert inf["vgprs"] > 0 and inf["scratch_bytes"] == 0 and inf["lds_bytes"] >= 0


def test_binding_rejects_argument_lists_of_the_wrong_length():
    import torch
    p = xg.Program(configs.program_path("rdag200"))
    x = torch.zeros((8, 4), dtype=torch.float64)
    with pytest.raises(xg.XgError, match="expected 1 input"):
        p.eval([x, x])
    with pytest.raises(xg.XgError, match="expected 1 seed"):
        p.eval_adjoint([x], [])
