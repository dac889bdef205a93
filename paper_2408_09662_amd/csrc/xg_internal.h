// Internal declarations of the xg library (not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "xg.h"

namespace xg {

// ---------------------------------------------------------------- IR
// SSA node.  Operands refer to earlier nodes (topological order).
// INPUT: aux = (arg << 32) | element.  CONST: aux = index into consts.
struct Node {
  uint8_t op;
  uint8_t f32 = 0;  // computed in binary32 inside an f64 program
  int32_t a = -1, b = -1;
  int64_t aux = 0;
};

struct Graph {
  int dtype = XG_F64;
  std::vector<int32_t> nnz_in, nnz_out;
  std::vector<double> consts;
  std::vector<Node> nodes;
  std::vector<std::vector<int32_t>> out;  // [arg][element] -> node id
};

bool is_binary(int op);
bool is_arith(int op);  // not INPUT/OUTPUT/CONST/ASSIGN
const char* op_name(int op);

// Validate the description, convert to SSA (slot reuse removed), merge
// common sub-expressions and drop dead code.
bool build_graph(const xg_program_desc& d, Graph& g, std::string& err);
// Remove nodes not reachable from the outputs and renumber (order kept).
void dce(Graph& g);
// Hash-consing pass (identical op + operands -> one node).
void cse(Graph& g);
// Divisions sharing a divisor (two or more, same precision) become one
// reciprocal and multiplications: a / b -> a * (1 / b).  Not exact (one
// more rounding); callers skip it in strict mode.  Returns the number of
// divisions replaced.
int64_t share_reciprocals(Graph& g);

// Reverse-mode adjoint as a program transformation.  The result's inputs
// are g's inputs followed by one seed argument per output of g (same
// sizes); its outputs are one gradient argument per input of g, followed by
// g's outputs if `with_primal`.  Ranges of more than `seg_ops` operations
// are cut into up to `fanout` parts at small live sets and reversed part by
// part from the states at the cuts (recursively); ranges of at most
// `seg_ops` operations are recomputed from the state at their start and
// then reversed (seg_ops <= 0: keep every value, no recomputation).
Graph adjoint(const Graph& g, bool with_primal, int seg_ops, int64_t* recompute_ops, int fanout = 4);

// ---------------------------------------------------------------- plan
struct Chunk {
  int32_t begin = 0, end = 0;  // range of the schedule
};

struct Plan {
  std::vector<int32_t> order;   // schedule: non-CONST node ids
  std::vector<Chunk> chunks;
  std::vector<int32_t> ws_slot; // per node: workspace slot (cross-chunk) or -1
  int32_t n_ws = 0;
  int64_t max_live = 0;
  int64_t n_ops = 0;
  // Cooperative tiles (waves > 1): W waves of one workgroup evaluate the
  // same 64 instances.  Chunk c runs on wave chunk_wave[c] in phase
  // chunk_phase[c]; phases are separated by a workgroup barrier, and every
  // value read by a chunk other than its own goes through the workspace.
  int32_t waves = 1;
  int32_t n_phases = 0;
  int32_t depth = 0;            // longest dependency chain (operations)
  std::vector<int32_t> chunk_phase, chunk_wave;
  // Phased cooperative tiles (narrow graphs): chunk w is everything wave w
  // computes, in order, across all phases; node_phase gives each node's
  // phase (a workgroup barrier separates consecutive phases inside every
  // wave's code), and a value read by another wave is stored once to the
  // LDS exchange slot xch_slot[v], read there after the barrier that ends
  // its phase.  Values stay in their wave's registers across phases.
  bool phased = false;
  std::vector<int32_t> node_phase, xch_slot;
  std::vector<int32_t> pos_phase;  // phase of each schedule position (a
                                   // cheap value may be computed by several
                                   // waves, in different phases)
  int32_t n_xch = 0;
  // mailbox[w * (n_phases + 1) + k]: other waves' values wave w copies
  // from their exchange slots right after the barrier that starts phase k
  std::vector<std::vector<int32_t>> mailbox;
  int64_t coop_est = 0;  // modelled time of the phased plan (cost units)
};

struct PlanOptions {
  int chunk_ops = 0;
  int waves = 1;
  int coop_phase = 0;  // > 0 with waves > 1: phased plan, this much work per wave and phase
  int64_t xch_cap = 0; // most LDS exchange slots the phased plan may use
};

// Relative issue cost of one operation (wave instructions, roughly).
int op_cost(int op);

Plan make_plan(const Graph& g, const PlanOptions& po);
int64_t max_live_of(const Graph& g, const std::vector<int32_t>& order);
// The non-CONST nodes in the order the planner prefers for register
// pressure: the front end's order or the greedy list schedule, whichever
// has the smaller maximum live set.
std::vector<int32_t> low_pressure_order(const Graph& g);

// ---------------------------------------------------------------- emit
struct EmitOptions {
  int block = 64;
  int ipt = 1;
  int reg_budget = 96;
  int lds_slots = 96;
  bool strict = false;
  bool call_math = true;  // branchy library functions as out-of-line calls
  int prefetch = 24;      // reloads are issued this many operations before use
  int waves = 1;          // > 1: cooperative tile (lane = threadIdx.x mod 64)
  bool inline_math = true; // SIN/COS inline and branch-free (else library calls)
};

struct EmitStats {
  int32_t lds_slots = 0;
  int32_t spills = 0;
  int32_t extra_ws = 0;  // global spill slots beyond LDS capacity
};

// Phased cooperative-tile program (plan.phased): one source, one kernel
// "<prefix>_c0" with the chunk kernels' signature, launched with 64 x waves
// lanes per workgroup and one workgroup per 64 instances.  The body is an
// if / else-if chain on the wave index, each branch holding that wave's
// whole share of the program with the phase barriers inline.
std::vector<std::string> emit_phased(const Graph& g, const Plan& plan, const EmitOptions& eo,
                                     const std::string& prefix, EmitStats* st);

// The same program as a function body for another kernel (the persistent
// batch): `body` needs n, ws, the argument pointers/pitches, ibase (the
// lane's instance: 64 x tile + lane), xg_w (the wave index) and
// xg_barrier() in scope, and addresses LDS from `lds_array`: the exchange
// slots, then one spill region per wave, lds_bytes in all.
struct PhasedParts {
  std::string body;
  int64_t ns = 0;         // workspace slots per instance
  int64_t lds_bytes = 0;
  EmitStats st;
};
PhasedParts emit_phased_parts(const Graph& g, const Plan& plan, const EmitOptions& eo,
                              const std::string& lds_array);

// One kernel per chunk.  Kernel c is named "<prefix>_c<c>", with the
// signature: (long long n, [const T* in_a, long long ld_in_a]...,
// [T* out_a, long long ld_out_a]..., T* ws).  The workspace holds, per
// block of block*ipt instances, [slot][ipt][block] elements.
// `extra_ws_base` is the first workspace slot free for global spills.
std::vector<std::string> emit_chunks(const Graph& g, const Plan& plan, const EmitOptions& eo,
                                     const std::string& prefix, EmitStats* st,
                                     int32_t extra_ws_base);

// Typedef of T, the access helpers and the math wrappers for g's dtype.
std::string emit_preamble(const Graph& g, const EmitOptions& eo);

// Body of chunk c as a noinline __device__ function `fname(long long
// ibase)` (used by the persistent batch kernel).  `prologue` must define
// n, ws, in<a>/ldi<a>, out<a>/ldo<a> and (if spills use LDS) lds; `ns`
// is the program's workspace slots per instance.
// Cooperative-tile program (plan.waves > 1): one source holding one
// kernel "<prefix>_c0" with the signature above, launched with
// 64 x waves threads per workgroup and one workgroup per 64 instances; its
// waves run the plan's chunks (noinline device functions) phase by phase
// with a workgroup barrier between phases.
std::vector<std::string> emit_wide(const Graph& g, const Plan& plan, const EmitOptions& eo,
                                   const std::string& prefix, EmitStats* st);

// The pieces of a cooperative-tile program for embedding in another kernel
// (the persistent batch): `funcs` defines one noinline device function per
// chunk ("<fprefix><c>"), each starting with `args_prologue` (which must
// define n, ws and the argument pointers/pitches); `body` runs the phases
// and needs `xg_w` (wave index in the workgroup) and `ibase` in scope.
struct WideParts {
  std::string funcs, body;
  int64_t ns = 0;              // workspace slots per instance
  int64_t lds_wave_elems = 0;  // LDS elements per wave
  EmitStats st;
};
WideParts emit_wide_parts(const Graph& g, const Plan& plan, const EmitOptions& eo,
                          const std::string& args_prologue, const std::string& lds_array,
                          const std::string& fprefix);

std::string emit_device_chunk(const Graph& g, const Plan& plan, int c, const EmitOptions& eo,
                              const std::string& fname, const std::string& prologue,
                              EmitStats* st, int32_t extra_ws_base, int64_t ns);

// ---------------------------------------------------------------- jit
struct CodeObject {
  std::vector<char> bin;
  double compile_ms = 0;
  bool cache_hit = false;
};
// Compile HIP source for gfx950 with hiprtc; served from the on-disk cache
// when the same source + options were compiled before.
bool compile_hip(const std::string& src, const std::vector<std::string>& opts, CodeObject& co,
                 std::string& err, bool verbose);
// Compile several sources, those missing from the cache in concurrent
// helper processes (the xg-rtc executable beside the library).
bool compile_many(const std::vector<std::string>& srcs, const std::vector<std::string>& opts,
                  std::vector<CodeObject>& cos, std::string& err, bool verbose);
std::vector<std::string> base_compile_options(bool strict);
// First line of a generated source: the FMA-contraction permission (none in
// strict mode).
std::string contract_pragma(bool strict);
// Resources of `kernel` from its kernel descriptor in the code object.
struct KernelDesc {
  uint32_t lds_bytes = 0;      // group segment (static LDS) per workgroup
  uint32_t scratch_bytes = 0;  // private segment per lane
  uint32_t kernarg_bytes = 0;  // argument segment, implicit arguments included
  int regs = 0;                // VGPRs + AGPRs per wave (granules of 8)
};
constexpr uint32_t kLdsBytesPerCU = 160 * 1024;
constexpr uint32_t kMaxScratchPerLane = 64 * 1024;
bool read_kernel_desc(const std::vector<char>& elf, const std::string& kernel, KernelDesc& kd);
// Registers (VGPRs + AGPRs) one wave of `kernel` uses; -1 if absent.
int kernel_vgprs(const std::vector<char>& elf, const std::string& kernel);
// Byte offset of the first implicit (hidden) kernel argument, from the code
// object's metadata note; -1 if absent.
int64_t kernel_hidden_args_offset(const std::vector<char>& elf, const std::string& kernel);
// False (with a message) if a `block`-lane workgroup of the kernel cannot be
// resident on one CU: registers per SIMD, LDS beyond 160 KiB, or scratch
// beyond kMaxScratchPerLane per lane.
bool check_launch_fits(const std::vector<char>& elf, const std::string& kernel, int block,
                       std::string& err);
// False (with a message) unless the kernel's implicit arguments start right
// after an explicit argument block of `explicit_bytes` bytes (rounded up to
// 8): kernels whose device functions find their argument block at that
// distance before the implicit-argument pointer rely on it.
bool check_kernel_args(const std::vector<char>& elf, const std::string& kernel, int64_t explicit_bytes,
                       std::string& err);
std::string cache_dir();
uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull);

void set_error(const std::string& e);

}  // namespace xg
