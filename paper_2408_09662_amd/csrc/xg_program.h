// Program object shared by the C-ABI implementation files.
#pragma once

#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "xg_internal.h"

namespace xg {

// LDS available to spill slots: 160 KiB per workgroup on gfx950 minus 512 B
// for a kernel's own shared variables (the batch kernel's job index).
constexpr int64_t kLdsSpillBytes = 160 * 1024 - 512;

struct DevMod {
  int device = -1;
  std::vector<hipModule_t> mods;
  std::vector<hipFunction_t> fns;
};

// One evaluation mode (0 forward, 1 adjoint, 2 fused forward + adjoint):
// its program, plan, generated sources and loaded code.
struct ModeState {
  bool planned = false;
  Graph g;
  Plan plan;
  EmitStats est;
  int64_t recompute_ops = 0;
  std::vector<std::string> srcs;
  std::vector<CodeObject> cos;
  bool compiled = false;
  bool checked = false;  // kernels checked against their launch (host only)
  double compile_ms = 0;
  int cache_hits = 0;
  std::vector<DevMod> devs;
  int32_t ws_slots() const { return plan.n_ws + est.extra_ws; }
};

// Workspace bytes for n instances: per block of block*ipt instances,
// ws_slots x block x ipt elements.
inline size_t ws_bytes_of(int64_t n, int32_t slots, int block, int ipt, size_t es) {
  const int64_t per = (int64_t)block * ipt;
  const int64_t tiles = (n + per - 1) / per;
  return (size_t)tiles * (size_t)slots * (size_t)per * es;
}

xg_options defaults(const xg_options* o, int dtype);
EmitOptions emit_options_of(const xg_options& o);
bool check_opts(const xg_options& o, int dtype, std::string& err);

}  // namespace xg

struct xg_program {
  xg::Graph g;
  xg_options opt;   // forward evaluation (mode 0)
  xg_options aopt;  // adjoint evaluations (modes 1 and 2); the load options until tuned
  xg::ModeState m[3];
  std::mutex mu;
  // HIP graphs whose kernel nodes run this program's loaded code.  While
  // any exists the code stays loaded: re-planning (autotuning) is refused
  // and xg_program_free only marks the program, which the last graph's
  // xg_graph_free then frees.
  int live_graphs = 0;
  bool free_pending = false;
};

// Options a mode is planned and launched with.
inline const xg_options& mode_opt(const xg_program* p, int mode) { return mode == 0 ? p->opt : p->aopt; }

namespace xg {
bool plan_mode(xg_program* p, int mode, std::string& err);
// hiprtc and host checks only (no device); *code as for compile_mode
bool build_code(xg_program* p, int mode, std::string& err, xg_status* code = nullptr);
// + load on the current device; on failure *code (if given) says why:
// XG_ECOMPILE, XG_EUNSUPPORTED (a kernel that cannot be launched as
// planned) or XG_EDEVICE
bool compile_mode(xg_program* p, int mode, std::string& err, xg_status* code = nullptr);
void reset_mode(xg_program* p, int mode);  // drain, unload, forget the plan
void destroy_program(xg_program* p);       // unload every mode and delete
// xg_eval_adjoint on the kernels already loaded on the current device, with
// a workspace of ws_cap bytes at ws; compiles, loads and allocates nothing
xg_status eval_adjoint_loaded(xg_program* p, int64_t n, const void* const* d_in, const int64_t* ld_in,
                              const void* const* d_out_bar, const int64_t* ld_out_bar,
                              void* const* d_out, const int64_t* ld_out, void* const* d_in_bar,
                              const int64_t* ld_in_bar, void* ws, size_t ws_cap, void* stream);
// device address of the fixed scratch array on the current device (looked
// up on the first call per device)
bool noalloc_scratch(void** ptr, std::string& err);
}  // namespace xg
