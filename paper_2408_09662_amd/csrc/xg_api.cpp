// The C ABI: program objects, planning, compilation, launches.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <map>
#include <memory>
#include <mutex>

#include <hip/hip_runtime.h>

#include "xg_internal.h"
#include "xg_program.h"

namespace xg {

static thread_local std::string g_err;
void set_error(const std::string& e) { g_err = e; }

}  // namespace xg

using namespace xg;

namespace xg {

xg_options defaults(const xg_options* o, int dtype) {
  xg_options d;
  std::memset(&d, 0, sizeof d);
  if (o) d = *o;
  if (d.waves <= 0) d.waves = 1;
  if (d.block <= 0) d.block = 64;
  if (d.ipt <= 0) d.ipt = 1;
  if (d.chunk_ops <= 0) d.chunk_ops = 20000;
  // 16-wave cooperative tiles put 4 waves on each SIMD: 128 registers each
  if (d.reg_budget <= 0) d.reg_budget = d.waves >= 16 ? (dtype == XG_F32 ? 96 : 48)
                                                      : (dtype == XG_F32 ? 200 : 112);
  if (d.lds_slots < 0) d.lds_slots = 0;
  // the plan allocates only the spill slots it needs, up to all 160 KiB
  if (d.lds_slots == 0)  // all of the 160 KiB but 512 B kept for the kernels' own variables
    d.lds_slots = (int32_t)(kLdsSpillBytes / ((int64_t)d.block * d.ipt * d.waves *
                                              (dtype == XG_F32 ? 4 : 8))) * d.ipt;
  if (d.adj_seg_ops == 0) d.adj_seg_ops = 250;
  if (d.adj_fanout <= 0) d.adj_fanout = 2;
  if (d.coop_phase < 0) d.coop_phase = 0;
  if (d.prefetch == 0) d.prefetch = 24;
  return d;
}

bool check_opts(const xg_options& o, int dtype, std::string& err) {
  if (o.block != 64 && o.block != 128 && o.block != 256 && o.block != 512 && o.block != 1024) {
    err = "block must be 64, 128, 256, 512 or 1024"; return false;
  }
  if (o.ipt != 1 && o.ipt != 2 && o.ipt != 4) { err = "ipt must be 1, 2 or 4"; return false; }
  if (o.inline_math < -1 || o.inline_math > 1) { err = "inline_math must be -1, 0 or 1"; return false; }
  if (o.adj_fanout < 2 || o.adj_fanout > 16) { err = "adj_fanout must be 2 ... 16"; return false; }
  if (o.waves != 1 && o.waves != 2 && o.waves != 4 && o.waves != 8 && o.waves != 16) {
    err = "waves must be 1, 2, 4, 8 or 16"; return false;
  }
  if (o.waves > 1 && (o.block != 64 || o.ipt != 1)) {
    err = "cooperative tiles (waves > 1) need block 64 and ipt 1"; return false;
  }
  // lds_slots counts per-lane slots of one element (ipt sub-slots per value),
  // per wave of a cooperative tile
  int64_t lds_bytes = (int64_t)o.lds_slots * o.block * o.waves * (dtype == XG_F32 ? 4 : 8);
  if (lds_bytes > kLdsSpillBytes) {
    err = "LDS spill area (lds_slots x block x element) exceeds 160 KiB - 512 B";
    return false;
  }
  return true;
}

EmitOptions emit_options_of(const xg_options& o) {
  EmitOptions eo;
  eo.block = o.block;
  eo.ipt = o.ipt;
  eo.reg_budget = o.reg_budget;
  eo.lds_slots = o.lds_slots;
  eo.strict = o.strict != 0;
  eo.prefetch = o.prefetch > 0 ? o.prefetch : 0;
  eo.waves = o.waves > 1 ? o.waves : 1;
  eo.inline_math = o.inline_math >= 0;
  return eo;
}

bool plan_mode(xg_program* p, int mode, std::string& err) {
  ModeState& M = p->m[mode];
  if (M.planned) return true;
  const xg_options& opt = mode_opt(p, mode);
  if (mode == 0) M.g = p->g;
  else M.g = adjoint(p->g, mode == 2, opt.adj_seg_ops, &M.recompute_ops, opt.adj_fanout);
  // outside strict mode, divisions by a shared divisor multiply by one
  // reciprocal (each saves the ~10-instruction IEEE division sequence)
  if (!opt.strict) share_reciprocals(M.g);
  PlanOptions po;
  po.chunk_ops = opt.chunk_ops;
  po.waves = mode == 0 ? opt.waves : 1;
  po.coop_phase = mode == 0 ? opt.coop_phase : 0;
  // exchange slots may take up to half of the LDS; spill slots get the rest
  po.xch_cap = kLdsSpillBytes / (64 * (M.g.dtype == XG_F32 ? 4 : 8)) / 2;
  try {
    M.plan = make_plan(M.g, po);
  } catch (const std::logic_error& e) {
    err = e.what();
    return false;
  }
  EmitOptions eo = emit_options_of(opt);
  eo.waves = M.plan.waves;
  char prefix[64];
  std::snprintf(prefix, sizeof prefix, "xg_m%d", mode);
  if (M.plan.phased) M.srcs = emit_phased(M.g, M.plan, eo, prefix, &M.est);
  else if (M.plan.waves > 1) M.srcs = emit_wide(M.g, M.plan, eo, prefix, &M.est);
  else M.srcs = emit_chunks(M.g, M.plan, eo, prefix, &M.est, M.plan.n_ws);
  if (opt.verbose)
    std::fprintf(stderr,
                 "[xg] mode %d: %zu nodes, %lld ops, max live %lld, %zu chunks, ws %d+%d slots, "
                 "lds %d slots, %d spills, recompute %lld, waves %d, phases %d, depth %d, xch %d, est %lld\n",
                 mode, M.g.nodes.size(), (long long)M.plan.n_ops, (long long)M.plan.max_live,
                 M.plan.chunks.size(), M.plan.n_ws, M.est.extra_ws, M.est.lds_slots, M.est.spills,
                 (long long)M.recompute_ops, M.plan.waves, M.plan.n_phases, M.plan.depth, M.plan.n_xch,
                 (long long)M.plan.coop_est);
  M.planned = true;
  (void)err;
  return true;
}

// Drop a mode's plan and code.  Kernels of it may still be queued or
// running (launches are asynchronous), so each device that holds its
// modules is drained before they are unloaded.
void reset_mode(xg_program* p, int mode) {
  ModeState& M = p->m[mode];
  bool loaded = false;
  for (auto& d : M.devs) loaded = loaded || !d.mods.empty();
  if (loaded) {  // no device call for code that was never loaded
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (auto& d : M.devs) {
      if (d.mods.empty()) continue;
      if (d.device >= 0 && hipSetDevice(d.device) == hipSuccess) (void)hipDeviceSynchronize();
      for (auto mod : d.mods) (void)hipModuleUnload(mod);
    }
    if (cur >= 0) (void)hipSetDevice(cur);
  }
  M = ModeState();
}

void destroy_program(xg_program* p) {
  for (int m = 0; m < 3; ++m) reset_mode(p, m);  // drains devices that hold its code
  delete p;
}

// Host checks of a mode's compiled kernels against the launch they get
// (no device needed): registers, LDS and scratch must let a workgroup be
// resident, and a cooperative tile's device functions must find the kernel
// arguments where they read them.
static bool check_mode_code(xg_program* p, int mode, std::string& err) {
  ModeState& M = p->m[mode];
  if (M.checked) return true;
  const int block = mode_opt(p, mode).block * M.plan.waves;
  for (size_t c = 0; c < M.cos.size(); ++c) {
    char name[64];
    std::snprintf(name, sizeof name, "xg_m%d_c%zu", mode, c);
    if (!check_launch_fits(M.cos[c].bin, name, block, err)) return false;
    // a cooperative tile reads the arguments (n, pointer/pitch pairs,
    // workspace) as one block placed just before the implicit arguments
    // (a phased tile reads its kernel arguments directly)
    if (M.plan.waves > 1 && !M.plan.phased &&
        !check_kernel_args(M.cos[c].bin, name, 8 * (2 + 2 * (int64_t)(M.g.nnz_in.size() + M.g.nnz_out.size())),
                           err))
      return false;
  }
  M.checked = true;
  return true;
}

bool build_code(xg_program* p, int mode, std::string& err, xg_status* code) {
  xg_status dummy;
  if (!code) code = &dummy;
  *code = XG_EINVAL;
  if (!plan_mode(p, mode, err)) return false;
  ModeState& M = p->m[mode];
  if (!M.compiled) {
    *code = XG_ECOMPILE;
    if (!compile_many(M.srcs, base_compile_options(mode_opt(p, mode).strict != 0), M.cos, err,
                      mode_opt(p, mode).verbose != 0))
      return false;
    M.compile_ms = 0;
    M.cache_hits = 0;
    for (auto& co : M.cos) { M.compile_ms += co.compile_ms; M.cache_hits += co.cache_hit; }
    M.compiled = true;
  }
  *code = XG_EUNSUPPORTED;
  return check_mode_code(p, mode, err);
}

bool compile_mode(xg_program* p, int mode, std::string& err, xg_status* code) {
  xg_status dummy;
  if (!code) code = &dummy;
  if (!build_code(p, mode, err, code)) return false;
  *code = XG_EDEVICE;
  ModeState& M = p->m[mode];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { err = "hipGetDevice failed"; return false; }
  for (auto& d : M.devs) if (d.device == dev) return true;
  // every kernel must fit its launch (code the autotuner compiled outside
  // build_code is checked here): a workgroup whose waves need more
  // registers than their SIMDs hold cannot be dispatched at all
  if (!check_mode_code(p, mode, err)) { *code = XG_EUNSUPPORTED; return false; }
  DevMod dm;
  dm.device = dev;
  auto unload = [&]() { for (auto mod : dm.mods) (void)hipModuleUnload(mod); };
  for (size_t c = 0; c < M.cos.size(); ++c) {
    hipModule_t mod;
    hipError_t e = hipModuleLoadData(&mod, M.cos[c].bin.data());
    if (e != hipSuccess) {
      unload();
      err = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
      return false;
    }
    dm.mods.push_back(mod);
    hipFunction_t f;
    char name[64];
    std::snprintf(name, sizeof name, "xg_m%d_c%zu", mode, c);
    e = hipModuleGetFunction(&f, mod, name);
    if (e != hipSuccess) {
      unload();
      err = std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
      return false;
    }
    dm.fns.push_back(f);
  }
  M.devs.push_back(dm);
  return true;
}

}  // namespace xg

namespace {

const DevMod* devmod(ModeState& M) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  for (auto& d : M.devs) if (d.device == dev) return &d;
  return nullptr;
}

size_t esize(const Graph& g) { return g.dtype == XG_F32 ? 4 : 8; }

bool check_args(const char* what, size_t nargs, const int32_t* nnz, const void* const* ptrs,
                const int64_t* ld, int64_t n, std::string& err) {
  for (size_t a = 0; a < nargs; ++a) {
    if (nnz[a] == 0) continue;
    if (!ptrs || !ptrs[a]) { err = std::string(what) + " pointer " + std::to_string(a) + " is null"; return false; }
    if (!ld || ld[a] < n) { err = std::string(what) + " pitch " + std::to_string(a) + " < n"; return false; }
  }
  return true;
}

struct Range { uintptr_t lo, hi; };

void ranges(size_t nargs, const int32_t* nnz, const void* const* ptrs, const int64_t* ld, int64_t n,
            size_t es, std::vector<Range>& out) {
  for (size_t a = 0; a < nargs; ++a) {
    if (nnz[a] == 0 || !ptrs || !ptrs[a]) continue;
    uintptr_t lo = (uintptr_t)ptrs[a];
    out.push_back({lo, lo + (uintptr_t)(((int64_t)(nnz[a] - 1) * ld[a] + n) * (int64_t)es)});
  }
}

bool overlap(const std::vector<Range>& A, const std::vector<Range>& B) {
  for (auto& a : A)
    for (auto& b : B)
      if (a.lo < b.hi && b.lo < a.hi) return true;
  return false;
}

xg_status launch_mode(xg_program* p, int mode, int64_t n, const std::vector<const void*>& in,
                      const std::vector<int64_t>& ldi, const std::vector<void*>& out,
                      const std::vector<int64_t>& ldo, void* ws, void* stream) {
  ModeState& M = p->m[mode];
  std::string err;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    xg_status code = XG_OK;
    if (!compile_mode(p, mode, err, &code)) {
      set_error(err);
      return code;
    }
  }
  const DevMod* dm = devmod(M);
  if (!dm) { set_error("module not loaded for current device"); return XG_EDEVICE; }
  if (M.ws_slots() > 0 && !ws) { set_error("this program needs a workspace (xg_workspace_bytes)"); return XG_EINVAL; }
  const xg_options& opt = mode_opt(p, mode);
  const int block = opt.block * M.plan.waves, ipt = opt.ipt;
  const int64_t per = (int64_t)opt.block * ipt;  // instances per workgroup
  const int64_t grid = (n + per - 1) / per;
  if (grid > INT32_MAX || (uint64_t)n * esize(M.g) > 0xffffffffull) {
    // lane byte offsets are 32-bit (the "SGPR base + VGPR offset" address form)
    set_error("n too large: n * sizeof(element) must stay below 4 GiB");
    return XG_EINVAL;
  }
  std::vector<uint64_t> st;
  st.reserve(4 + 2 * (in.size() + out.size()));
  st.push_back((uint64_t)n);
  for (size_t a = 0; a < in.size(); ++a) { st.push_back((uint64_t)(uintptr_t)in[a]); st.push_back((uint64_t)ldi[a]); }
  for (size_t a = 0; a < out.size(); ++a) { st.push_back((uint64_t)(uintptr_t)out[a]); st.push_back((uint64_t)ldo[a]); }
  st.push_back((uint64_t)(uintptr_t)ws);
  std::vector<void*> params(st.size());
  for (size_t i = 0; i < st.size(); ++i) params[i] = &st[i];
  for (size_t c = 0; c < dm->fns.size(); ++c) {
    hipError_t e = hipModuleLaunchKernel(dm->fns[c], (unsigned)grid, 1, 1, (unsigned)block, 1, 1, 0,
                                         (hipStream_t)stream, params.data(), nullptr);
    if (e != hipSuccess) {
      set_error(std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
      return XG_EDEVICE;
    }
  }
  return XG_OK;
}

}  // namespace

namespace xg {

// xg_eval_adjoint on kernels already loaded on the current device, with a
// workspace of ws_cap bytes at ws: compiles nothing, loads nothing and
// allocates no memory (argument checks and the launch use stack arrays).
xg_status eval_adjoint_loaded(xg_program* p, int64_t n, const void* const* d_in, const int64_t* ld_in,
                              const void* const* d_out_bar, const int64_t* ld_out_bar,
                              void* const* d_out, const int64_t* ld_out, void* const* d_in_bar,
                              const int64_t* ld_in_bar, void* ws, size_t ws_cap, void* stream) {
  if (!p) { set_error("program is null"); return XG_EINVAL; }
  if (n < 0) { set_error("n < 0"); return XG_EINVAL; }
  if (n == 0) return XG_OK;
  const Graph& g = p->g;
  const size_t nin = g.nnz_in.size(), nout = g.nnz_out.size();
  constexpr size_t kMaxArgs = 64;  // pointer/pitch pairs of one launch
  if (2 * (nin + nout) > kMaxArgs) {
    set_error("more arguments than this entry point passes (64 pointer/pitch pairs)");
    return XG_EUNSUPPORTED;
  }
  const size_t es = esize(g);
  // argument checks as xg_eval_adjoint's, on fixed-size arrays
  Range ri[kMaxArgs], ro[kMaxArgs];
  size_t nri = 0, nro = 0;
  struct ArgList { const char* what; size_t k; const int32_t* nnz; const void* const* ptr; const int64_t* ld; bool in; };
  const ArgList lists[4] = {
      {"input", nin, g.nnz_in.data(), d_in, ld_in, true},
      {"seed", nout, g.nnz_out.data(), d_out_bar, ld_out_bar, true},
      {"gradient", nin, g.nnz_in.data(), (const void* const*)d_in_bar, ld_in_bar, false},
      {"output", d_out ? nout : 0, g.nnz_out.data(), (const void* const*)d_out, ld_out, false}};
  for (const ArgList& L : lists) {
    for (size_t a = 0; a < L.k; ++a) {
      if (L.nnz[a] == 0) continue;
      if (!L.ptr || !L.ptr[a]) {
        char m[96];
        std::snprintf(m, sizeof m, "%s pointer %zu is null", L.what, a);
        set_error(m);
        return XG_EINVAL;
      }
      if (!L.ld || L.ld[a] < n) {
        char m[96];
        std::snprintf(m, sizeof m, "%s pitch %zu < n", L.what, a);
        set_error(m);
        return XG_EINVAL;
      }
      const uintptr_t lo = (uintptr_t)L.ptr[a];
      const Range r{lo, lo + (uintptr_t)(((int64_t)(L.nnz[a] - 1) * L.ld[a] + n) * (int64_t)es)};
      if (L.in) ri[nri++] = r; else ro[nro++] = r;
    }
  }
  for (size_t i = 0; i < nri; ++i)
    for (size_t j = 0; j < nro; ++j)
      if (ri[i].lo < ro[j].hi && ro[j].lo < ri[i].hi) { set_error("an output overlaps an input"); return XG_EALIAS; }
  const int mode = d_out ? 2 : 1;
  ModeState& M = p->m[mode];
  // the kernel handles are copied under the lock (another thread may load
  // the mode on another device meanwhile, which grows the module table)
  constexpr size_t kMaxKernels = 64;
  hipFunction_t fns[kMaxKernels];
  size_t n_fns = 0;
  int block = 0, ipt = 1, per = 0;
  int32_t slots = 0;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    const DevMod* dm = M.compiled ? devmod(M) : nullptr;
    if (dm && dm->fns.size() > kMaxKernels) {
      set_error("more kernels per evaluation than this entry point launches (64)");
      return XG_EUNSUPPORTED;
    }
    if (dm) {
      n_fns = dm->fns.size();
      for (size_t c = 0; c < n_fns; ++c) fns[c] = dm->fns[c];
    }
    if (!dm) {
      set_error(mode == 2 ? "the fused adjoint (mode 2) is not loaded on this device: call xg_compile(p, 2) first"
                          : "the adjoint (mode 1) is not loaded on this device: call xg_compile(p, 1) first");
      return XG_EINVAL;
    }
    const xg_options& opt = mode_opt(p, mode);
    block = opt.block * M.plan.waves;
    ipt = opt.ipt;
    per = opt.block * ipt;
    slots = M.ws_slots();
  }
  const int64_t grid = (n + per - 1) / per;
  if (grid > INT32_MAX || (uint64_t)n * es > 0xffffffffull) {
    set_error("n too large: n * sizeof(element) must stay below 4 GiB");
    return XG_EINVAL;
  }
  const size_t need = ws_bytes_of(n, slots, per / ipt, ipt, es);
  if (need > ws_cap) {
    char m[200];
    std::snprintf(m, sizeof m,
                  "%lld instances need %zu bytes of workspace; the fixed scratch array holds %zu "
                  "(use xg_eval_adjoint with a caller-provided workspace)",
                  (long long)n, need, ws_cap);
    set_error(m);
    return XG_ENOMEM;
  }
  uint64_t st[2 + 2 * 2 * kMaxArgs];
  size_t k = 0;
  st[k++] = (uint64_t)n;
  for (size_t a = 0; a < nin; ++a) { st[k++] = (uint64_t)(uintptr_t)d_in[a]; st[k++] = (uint64_t)ld_in[a]; }
  for (size_t a = 0; a < nout; ++a) { st[k++] = (uint64_t)(uintptr_t)d_out_bar[a]; st[k++] = (uint64_t)ld_out_bar[a]; }
  for (size_t a = 0; a < nin; ++a) { st[k++] = (uint64_t)(uintptr_t)d_in_bar[a]; st[k++] = (uint64_t)ld_in_bar[a]; }
  if (d_out)
    for (size_t a = 0; a < nout; ++a) { st[k++] = (uint64_t)(uintptr_t)d_out[a]; st[k++] = (uint64_t)ld_out[a]; }
  st[k++] = (uint64_t)(uintptr_t)ws;
  void* params[2 + 2 * 2 * kMaxArgs];
  for (size_t i = 0; i < k; ++i) params[i] = &st[i];
  for (size_t c = 0; c < n_fns; ++c) {
    hipError_t e = hipModuleLaunchKernel(fns[c], (unsigned)grid, 1, 1, (unsigned)block, 1, 1, 0,
                                         (hipStream_t)stream, params, nullptr);
    if (e != hipSuccess) {
      set_error(std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
      return XG_EDEVICE;
    }
  }
  return XG_OK;
}

}  // namespace xg

extern "C" {

const char* xg_last_error(void) { return g_err.c_str(); }
const char* xg_version(void) { return "xg 0.1 (gfx950)"; }

xg_status xg_program_load(const xg_program_desc* desc, const xg_options* opts, xg_program** out) {
  if (!out) { set_error("out is null"); return XG_EINVAL; }
  *out = nullptr;
  if (!desc) { set_error("desc is null"); return XG_EINVAL; }
  std::unique_ptr<xg_program> p(new (std::nothrow) xg_program());
  if (!p) { set_error("out of host memory"); return XG_ENOMEM; }
  std::string err;
  try {
    if (!build_graph(*desc, p->g, err)) { set_error(err); return XG_EINVAL; }
    p->opt = defaults(opts, desc->dtype);
    if (!check_opts(p->opt, desc->dtype, err)) { set_error(err); return XG_EINVAL; }
    p->aopt = p->opt;
    if (p->opt.eager) {
      if (!plan_mode(p.get(), 0, err) || !compile_mode(p.get(), 0, err)) {
        set_error(err);
        return XG_ECOMPILE;
      }
    }
  } catch (const std::bad_alloc&) {
    set_error("out of host memory");
    return XG_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return XG_EINVAL;
  }
  *out = p.release();
  return XG_OK;
}

void xg_program_free(xg_program* p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->live_graphs > 0) {  // graphs still launch its kernels: the last one frees it
      p->free_pending = true;
      return;
    }
  }
  destroy_program(p);
}

xg_status xg_program_options(xg_program* p, int32_t mode, xg_options* out) {
  if (!p || !out || mode < 0 || mode > 2) { set_error("bad argument"); return XG_EINVAL; }
  std::lock_guard<std::mutex> lk(p->mu);
  *out = mode_opt(p, mode);
  return XG_OK;
}

xg_status xg_program_info(xg_program* p, int32_t mode, xg_info* info) {
  if (!p || !info || mode < 0 || mode > 2) { set_error("bad argument"); return XG_EINVAL; }
  std::string err;
  std::lock_guard<std::mutex> lk(p->mu);
  try {
    if (!plan_mode(p, mode, err)) { set_error(err); return XG_EINVAL; }
  } catch (const std::exception& e) { set_error(e.what()); return XG_ENOMEM; }
  ModeState& M = p->m[mode];
  std::memset(info, 0, sizeof *info);
  info->n_nodes = (int64_t)M.g.nodes.size();
  info->n_ops = M.plan.n_ops;
  info->max_live = M.plan.max_live;
  info->n_chunks = (int32_t)M.srcs.size();  // kernels per evaluation
  info->n_ws_slots = M.ws_slots();
  info->n_lds_slots = M.est.lds_slots;
  info->n_spills = M.est.spills;
  info->compile_ms = M.compile_ms;
  info->cache_hits = M.cache_hits;
  info->vgprs = 0;
  for (size_t c = 0; c < M.cos.size(); ++c) {  // once compiled: from the kernel descriptors
    char name[64];
    std::snprintf(name, sizeof name, "xg_m%d_c%zu", mode, c);
    KernelDesc kd;
    if (!read_kernel_desc(M.cos[c].bin, name, kd)) continue;
    info->vgprs = std::max(info->vgprs, (int32_t)kd.regs);
    info->lds_bytes = std::max(info->lds_bytes, (int32_t)kd.lds_bytes);
    info->scratch_bytes = std::max(info->scratch_bytes, (int32_t)kd.scratch_bytes);
  }
  uint64_t h = 1469598103934665603ull;
  for (const auto& o : base_compile_options(mode_opt(p, mode).strict != 0)) h = fnv1a(o, h);
  for (const auto& src : M.srcs) h = fnv1a(src, h);
  info->code_hash = h;
  return XG_OK;
}

xg_status xg_workspace_bytes(xg_program* p, int64_t n, int32_t mode, size_t* bytes) {
  if (!p || !bytes || n < 0 || mode < 0 || mode > 2) { set_error("bad argument"); return XG_EINVAL; }
  std::string err;
  std::lock_guard<std::mutex> lk(p->mu);
  try {
    if (!plan_mode(p, mode, err)) { set_error(err); return XG_EINVAL; }
  } catch (const std::exception& e) { set_error(e.what()); return XG_ENOMEM; }
  ModeState& M = p->m[mode];
  *bytes = ws_bytes_of(n, M.ws_slots(), mode_opt(p, mode).block, mode_opt(p, mode).ipt, esize(M.g));
  return XG_OK;
}

xg_status xg_precompile(xg_program* p, int32_t mode) {
  if (!p || mode < 0 || mode > 2) { set_error("bad argument"); return XG_EINVAL; }
  std::string err;
  std::lock_guard<std::mutex> lk(p->mu);
  try {
    xg_status code = XG_OK;
    if (!build_code(p, mode, err, &code)) { set_error(err); return code; }
  } catch (const std::exception& e) { set_error(e.what()); return XG_ENOMEM; }
  return XG_OK;
}

xg_status xg_compile(xg_program* p, int32_t mode) {
  if (!p || mode < 0 || mode > 2) { set_error("bad argument"); return XG_EINVAL; }
  std::string err;
  std::lock_guard<std::mutex> lk(p->mu);
  try {
    xg_status code = XG_OK;
    if (!compile_mode(p, mode, err, &code)) { set_error(err); return code; }
  } catch (const std::exception& e) { set_error(e.what()); return XG_ENOMEM; }
  return XG_OK;
}

xg_status xg_eval(xg_program* p, int64_t n, const void* const* d_in, const int64_t* ld_in,
                  void* const* d_out, const int64_t* ld_out, void* d_workspace, void* stream) {
  if (!p) { set_error("program is null"); return XG_EINVAL; }
  if (n < 0) { set_error("n < 0"); return XG_EINVAL; }
  if (n == 0) return XG_OK;
  const Graph& g = p->g;
  std::string err;
  if (!check_args("input", g.nnz_in.size(), g.nnz_in.data(), d_in, ld_in, n, err) ||
      !check_args("output", g.nnz_out.size(), g.nnz_out.data(), (const void* const*)d_out, ld_out, n, err)) {
    set_error(err);
    return XG_EINVAL;
  }
  std::vector<Range> ri, ro;
  ranges(g.nnz_in.size(), g.nnz_in.data(), d_in, ld_in, n, esize(g), ri);
  ranges(g.nnz_out.size(), g.nnz_out.data(), (const void* const*)d_out, ld_out, n, esize(g), ro);
  if (overlap(ri, ro)) { set_error("an output overlaps an input"); return XG_EALIAS; }
  std::vector<const void*> in(g.nnz_in.size());
  std::vector<int64_t> ldi(g.nnz_in.size());
  for (size_t a = 0; a < in.size(); ++a) { in[a] = d_in ? d_in[a] : nullptr; ldi[a] = ld_in ? ld_in[a] : n; }
  std::vector<void*> out(g.nnz_out.size());
  std::vector<int64_t> ldo(g.nnz_out.size());
  for (size_t a = 0; a < out.size(); ++a) { out[a] = d_out ? d_out[a] : nullptr; ldo[a] = ld_out ? ld_out[a] : n; }
  try {
    return launch_mode(p, 0, n, in, ldi, out, ldo, d_workspace, stream);
  } catch (const std::exception& e) { set_error(e.what()); return XG_ENOMEM; }
}

xg_status xg_eval_adjoint(xg_program* p, int64_t n, const void* const* d_in, const int64_t* ld_in,
                          const void* const* d_out_bar, const int64_t* ld_out_bar,
                          void* const* d_out, const int64_t* ld_out, void* const* d_in_bar,
                          const int64_t* ld_in_bar, void* d_workspace, void* stream) {
  if (!p) { set_error("program is null"); return XG_EINVAL; }
  if (n < 0) { set_error("n < 0"); return XG_EINVAL; }
  if (n == 0) return XG_OK;
  const Graph& g = p->g;
  std::string err;
  if (!check_args("input", g.nnz_in.size(), g.nnz_in.data(), d_in, ld_in, n, err) ||
      !check_args("seed", g.nnz_out.size(), g.nnz_out.data(), d_out_bar, ld_out_bar, n, err) ||
      !check_args("gradient", g.nnz_in.size(), g.nnz_in.data(), (const void* const*)d_in_bar, ld_in_bar, n, err) ||
      (d_out && !check_args("output", g.nnz_out.size(), g.nnz_out.data(), (const void* const*)d_out, ld_out, n, err))) {
    set_error(err);
    return XG_EINVAL;
  }
  std::vector<Range> ri, ro;
  ranges(g.nnz_in.size(), g.nnz_in.data(), d_in, ld_in, n, esize(g), ri);
  ranges(g.nnz_out.size(), g.nnz_out.data(), d_out_bar, ld_out_bar, n, esize(g), ri);
  ranges(g.nnz_in.size(), g.nnz_in.data(), (const void* const*)d_in_bar, ld_in_bar, n, esize(g), ro);
  if (d_out) ranges(g.nnz_out.size(), g.nnz_out.data(), (const void* const*)d_out, ld_out, n, esize(g), ro);
  if (overlap(ri, ro)) { set_error("an output overlaps an input"); return XG_EALIAS; }
  const int mode = d_out ? 2 : 1;
  std::vector<const void*> in;
  std::vector<int64_t> ldi;
  for (size_t a = 0; a < g.nnz_in.size(); ++a) { in.push_back(d_in[a]); ldi.push_back(ld_in[a]); }
  for (size_t a = 0; a < g.nnz_out.size(); ++a) { in.push_back(d_out_bar[a]); ldi.push_back(ld_out_bar[a]); }
  std::vector<void*> out;
  std::vector<int64_t> ldo;
  for (size_t a = 0; a < g.nnz_in.size(); ++a) { out.push_back(d_in_bar[a]); ldo.push_back(ld_in_bar[a]); }
  if (d_out)
    for (size_t a = 0; a < g.nnz_out.size(); ++a) { out.push_back(d_out[a]); ldo.push_back(ld_out[a]); }
  try {
    return launch_mode(p, mode, n, in, ldi, out, ldo, d_workspace, stream);
  } catch (const std::exception& e) { set_error(e.what()); return XG_ENOMEM; }
}

}  // extern "C"
