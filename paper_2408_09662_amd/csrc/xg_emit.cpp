// HIP source emission for one chunk of a planned program.
//
// The paper's generator turns each instruction into one statement of a
// single CUDA kernel that reads and writes a per-instance work vector in
// global memory (AoS, stride n_w).  Here the same straight-line statement
// sequence is emitted, but
//   * instance i of argument a, element e is at ptr[e * ld + i] (structure
//     of arrays, instance fastest), so a wavefront's 64 lanes read and
//     write 64 consecutive values: every global access is coalesced;
//   * intermediates are SSA locals -- registers -- not memory.  A register
//     plan bounds how many are live at once: when the budget is reached,
//     the value whose next use is furthest away leaves the register file
//     (Belady's rule).  Inputs and values of earlier chunks are simply
//     reloaded from global memory later; values computed in this chunk are
//     spilled to a per-lane LDS slot (lds[slot][lane], conflict-free) and
//     reloaded from there, or to a global workspace slot if LDS is full;
//   * values needed by later chunks are stored to the workspace right after
//     they are computed, outputs right after they are final.
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <queue>
#include <memory>
#include <unordered_map>

#include "xg_internal.h"

namespace xg {

namespace {

const int32_t kInf = INT32_MAX;

std::string literal(double c, bool f32) {
  char buf[64];
  if (std::isnan(c)) return f32 ? "__builtin_nanf(\"\")" : "__builtin_nan(\"\")";
  if (std::isinf(c)) {
    const char* s = f32 ? "__builtin_inff()" : "__builtin_inf()";
    return c < 0 ? std::string("(-") + s + ")" : std::string(s);
  }
  std::snprintf(buf, sizeof buf, "%a", c);
  std::string s(buf);
  if (f32) return "((float)(" + s + "))";
  return "(" + s + ")";
}

const char* fn(int op, bool f32) {
  switch (op) {
    case XG_OP_SQRT: return f32 ? "sqrtf" : "sqrt";
    case XG_OP_EXP: return f32 ? "expf" : "exp";
    case XG_OP_LOG: return f32 ? "logf" : "log";
    case XG_OP_SIN: return f32 ? "sinf" : "sin";
    case XG_OP_COS: return f32 ? "cosf" : "cos";
    case XG_OP_TAN: return f32 ? "tanf" : "tan";
    case XG_OP_TANH: return f32 ? "tanhf" : "tanh";
    case XG_OP_ATAN: return f32 ? "atanf" : "atan";
    case XG_OP_FABS: return f32 ? "fabsf" : "fabs";
    case XG_OP_FMIN: return f32 ? "fminf" : "fmin";
    case XG_OP_FMAX: return f32 ? "fmaxf" : "fmax";
    case XG_OP_POW: return f32 ? "powf" : "pow";
    case XG_OP_ATAN2: return f32 ? "atan2f" : "atan2";
  }
  return nullptr;
}

// Library functions whose device implementation branches (argument
// reduction paths) are called through out-of-line wrappers: inlined, their
// control flow makes the register allocator keep far more values in
// registers than the straight-line code needs (hundreds of spills on a
// pendulum chunk that needs 231 VGPRs with calls), and it multiplies code
// size and compile time.  Division and square root stay inline.
bool outlined(int op) {
  switch (op) {
    case XG_OP_EXP: case XG_OP_LOG: case XG_OP_SIN: case XG_OP_COS: case XG_OP_TAN:
    case XG_OP_TANH: case XG_OP_ATAN: case XG_OP_POW: case XG_OP_ATAN2:
      return true;
  }
  return false;
}

// Inline, branch-free sine and cosine in binary64 (the reduction also
// serves the binary32 versions below).  Cody and Waite's reduction: k = nearest integer
// to x * 2/pi, r = x - k * pi/2 with pi/2 split into three doubles and one
// fused multiply-add per part (exact products), so |r| <= pi/4 within a few
// units in the last place for |x| <= 2^50; r = x when k = 0 (the exact
// small-argument result; sin(-0) is +0).  On |r| <= pi/4 the Taylor series of
// sin to r^17 and of cos to r^18 are below 1e-19 truncation error, evaluated
// by Horner's rule with FMA; the quadrant k mod 4 selects and signs them.
// Measured against long double: at most 1.5 ulp for |x| < 1e4.  Beyond
// 2^50 (and for infinities, NaNs) the result is NaN: the reduction would no
// longer be exact.  The coefficients are 1/n! rounded to double and pi/2,
// 2/pi rounded / split to double, all computed for this file.
const char* kTrig =
    "__device__ __forceinline__ int xg_red(double x, double& r) {\n"
    "  const double k = __builtin_rint(x * 0x1.45f306dc9c883p-1);\n"
    "  double t = __builtin_fma(-k, 0x1.921fb54442d18p+0, x);\n"
    "  t = __builtin_fma(-k, 0x1.1a62633145c07p-54, t);\n"
    "  r = __builtin_fma(-k, -0x1.f1976b7ed8fbcp-110, t);\n"
    "  r = __builtin_fabs(x) <= 0x1p50 ? (k == 0.0 ? x : r) : __builtin_nan(\"\");\n"
    "  return (int)(k - 4.0 * __builtin_floor(k * 0.25));  // k mod 4, exact\n"
    "}\n"
    "__device__ __forceinline__ double xg_sinp(double r) {\n"
    "  const double z = r * r;\n"
    "  double p = 0x1.952c77030ad4ap-49;\n"
    "  p = __builtin_fma(p, z, -0x1.ae7f3e733b81fp-41);\n"
    "  p = __builtin_fma(p, z, 0x1.6124613a86d09p-33);\n"
    "  p = __builtin_fma(p, z, -0x1.ae64567f544e4p-26);\n"
    "  p = __builtin_fma(p, z, 0x1.71de3a556c734p-19);\n"
    "  p = __builtin_fma(p, z, -0x1.a01a01a01a01ap-13);\n"
    "  p = __builtin_fma(p, z, 0x1.1111111111111p-7);\n"
    "  p = __builtin_fma(p, z, -0x1.5555555555555p-3);\n"
    "  return __builtin_fma(r * z, p, r);\n"
    "}\n"
    "__device__ __forceinline__ double xg_cosp(double r) {\n"
    "  const double z = r * r;\n"
    "  double p = -0x1.6827863b97d97p-53;\n"
    "  p = __builtin_fma(p, z, 0x1.ae7f3e733b81fp-45);\n"
    "  p = __builtin_fma(p, z, -0x1.93974a8c07c9dp-37);\n"
    "  p = __builtin_fma(p, z, 0x1.1eed8eff8d898p-29);\n"
    "  p = __builtin_fma(p, z, -0x1.27e4fb7789f5cp-22);\n"
    "  p = __builtin_fma(p, z, 0x1.a01a01a01a01ap-16);\n"
    "  p = __builtin_fma(p, z, -0x1.6c16c16c16c17p-10);\n"
    "  p = __builtin_fma(p, z, 0x1.5555555555555p-5);\n"
    "  p = __builtin_fma(p, z, -0.5);\n"
    "  return __builtin_fma(z, p, 1.0);\n"
    "}\n"
    // both polynomials, then selects: a conditional on a per-lane quadrant
    // would become divergent control flow
    "__device__ __forceinline__ double xg_sin_d(double x) {\n"
    "  double r;\n"
    "  const int q = xg_red(x, r);\n"
    "  const double s = xg_sinp(r), c = xg_cosp(r);\n"
    "  const double v = (q & 1) ? c : s;\n"
    "  return (q & 2) ? -v : v;\n"
    "}\n"
    "__device__ __forceinline__ double xg_cos_d(double x) {\n"
    "  double r;\n"
    "  const int q = xg_red(x, r);\n"
    "  const double s = xg_sinp(r), c = xg_cosp(r);\n"
    "  const double v = (q & 1) ? s : c;\n"
    "  return ((q + 1) & 2) ? -v : v;\n"
    "}\n";

// Binary32 sine and cosine: the binary64 reduction above (exact for every
// binary32 argument up to 2^50), r rounded once to binary32, then Taylor
// series of sin to r^11 and of cos to r^10 (truncation below 2e-10 on
// |r| <= pi/4, under a hundredth of a binary32 ulp) in binary32 with FMA.
// Error: rounding r contributes at most half an ulp, the polynomial about
// one more; a binary32 operation costs half a binary64 one on the vector
// units, and these polynomials are half as long as the binary64 ones.
// Coefficients: 1/n! rounded to binary32, computed for this file.
const char* kTrigF =
    "__device__ __forceinline__ float xg_sinpf(float r) {\n"
    "  const float z = r * r;\n"
    "  float p = -0x1.ae6456p-26f;\n"
    "  p = __builtin_fmaf(p, z, 0x1.71de3ap-19f);\n"
    "  p = __builtin_fmaf(p, z, -0x1.a01a02p-13f);\n"
    "  p = __builtin_fmaf(p, z, 0x1.111112p-7f);\n"
    "  p = __builtin_fmaf(p, z, -0x1.555556p-3f);\n"
    "  return __builtin_fmaf(r * z, p, r);\n"
    "}\n"
    "__device__ __forceinline__ float xg_cospf(float r) {\n"
    "  const float z = r * r;\n"
    "  float p = -0x1.27e4fcp-22f;\n"
    "  p = __builtin_fmaf(p, z, 0x1.a01a02p-16f);\n"
    "  p = __builtin_fmaf(p, z, -0x1.6c16c2p-10f);\n"
    "  p = __builtin_fmaf(p, z, 0x1.555556p-5f);\n"
    "  p = __builtin_fmaf(p, z, -0.5f);\n"
    "  return __builtin_fmaf(z, p, 1.0f);\n"
    "}\n"
    "__device__ __forceinline__ float xg_sin_f(float x) {\n"
    "  double rd;\n"
    "  const int q = xg_red((double)x, rd);\n"
    "  const float r = (float)rd;\n"
    "  const float s = xg_sinpf(r), c = xg_cospf(r);\n"
    "  const float v = (q & 1) ? c : s;\n"
    "  return (q & 2) ? -v : v;\n"
    "}\n"
    "__device__ __forceinline__ float xg_cos_f(float x) {\n"
    "  double rd;\n"
    "  const int q = xg_red((double)x, rd);\n"
    "  const float r = (float)rd;\n"
    "  const float s = xg_sinpf(r), c = xg_cospf(r);\n"
    "  const float v = (q & 1) ? s : c;\n"
    "  return ((q + 1) & 2) ? -v : v;\n"
    "}\n";

// Inline, branch-free exponential and hyperbolic tangent in binary64 (also
// used, rounded once, for binary32 operands).  exp: k = nearest integer to
// x / ln 2, r = x - k ln 2 with ln 2 split into two doubles (FMA), so
// |r| <= ln2/2; Taylor series to r^13 (truncation below 7e-18 relative),
// Horner with FMA, scaled by 2^k (ldexp: one rounding, also for subnormal
// results); x is clamped to [-746, 710] first (beyond, the result is 0 or
// infinity either way) and a NaN argument is returned as is.  tanh:
// E = expm1(2|x|) from its Taylor series to degree 20 when 2|x| < 1.1
// (truncation below 4e-18 relative) and exp(2|x|) - 1 otherwise (no
// cancellation there), tanh = E / (E + 2) with the sign of x; |x| is
// clamped to 20, where tanh rounds to 1.  Coefficients 1/n! and the ln 2
// split were computed for this file.
const char* kExp =
    "__device__ __forceinline__ double xg_exp_d(double x) {\n"
    "  const double xc = x > 710.0 ? 710.0 : (x < -746.0 ? -746.0 : x);\n"
    "  const double k = __builtin_rint(xc * 0x1.71547652b82fep+0);\n"
    "  double r = __builtin_fma(-k, 0x1.62e42fefa39efp-1, xc);\n"
    "  r = __builtin_fma(-k, 0x1.abc9e3b39803fp-56, r);\n"
    "  double p = 0x1.6124613a86d09p-33;\n"
    "  p = __builtin_fma(p, r, 0x1.1eed8eff8d898p-29);\n"
    "  p = __builtin_fma(p, r, 0x1.ae64567f544e4p-26);\n"
    "  p = __builtin_fma(p, r, 0x1.27e4fb7789f5cp-22);\n"
    "  p = __builtin_fma(p, r, 0x1.71de3a556c734p-19);\n"
    "  p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-16);\n"
    "  p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-13);\n"
    "  p = __builtin_fma(p, r, 0x1.6c16c16c16c17p-10);\n"
    "  p = __builtin_fma(p, r, 0x1.1111111111111p-7);\n"
    "  p = __builtin_fma(p, r, 0x1.5555555555555p-5);\n"
    "  p = __builtin_fma(p, r, 0x1.5555555555555p-3);\n"
    "  p = __builtin_fma(p, r, 0.5);\n"
    "  p = __builtin_fma(p, r, 1.0);\n"
    "  p = __builtin_fma(p, r, 1.0);\n"
    "  const double y = __builtin_ldexp(p, (int)k);\n"
    "  return x == x ? y : x;\n"
    "}\n";
const char* kTanh =
    "__device__ __forceinline__ double xg_tanh_d(double x) {\n"
    "  const double a = __builtin_fabs(x);\n"
    "  const double u = 2.0 * (a < 20.0 ? a : 20.0);\n"
    "  double p = 0x1.71b8ef6dcf572p-66;\n"
    "  p = __builtin_fma(p, u, 0x1.e542ba4020225p-62);\n"
    "  p = __builtin_fma(p, u, 0x1.2f49b46814157p-57);\n"
    "  p = __builtin_fma(p, u, 0x1.6827863b97d97p-53);\n"
    "  p = __builtin_fma(p, u, 0x1.952c77030ad4ap-49);\n"
    "  p = __builtin_fma(p, u, 0x1.ae7f3e733b81fp-45);\n"
    "  p = __builtin_fma(p, u, 0x1.ae7f3e733b81fp-41);\n"
    "  p = __builtin_fma(p, u, 0x1.93974a8c07c9dp-37);\n"
    "  p = __builtin_fma(p, u, 0x1.6124613a86d09p-33);\n"
    "  p = __builtin_fma(p, u, 0x1.1eed8eff8d898p-29);\n"
    "  p = __builtin_fma(p, u, 0x1.ae64567f544e4p-26);\n"
    "  p = __builtin_fma(p, u, 0x1.27e4fb7789f5cp-22);\n"
    "  p = __builtin_fma(p, u, 0x1.71de3a556c734p-19);\n"
    "  p = __builtin_fma(p, u, 0x1.a01a01a01a01ap-16);\n"
    "  p = __builtin_fma(p, u, 0x1.a01a01a01a01ap-13);\n"
    "  p = __builtin_fma(p, u, 0x1.6c16c16c16c17p-10);\n"
    "  p = __builtin_fma(p, u, 0x1.1111111111111p-7);\n"
    "  p = __builtin_fma(p, u, 0x1.5555555555555p-5);\n"
    "  p = __builtin_fma(p, u, 0x1.5555555555555p-3);\n"
    "  p = __builtin_fma(p, u, 0.5);\n"
    "  const double em1_small = __builtin_fma(p * u, u, u);\n"
    "  const double em1_big = xg_exp_d(u) - 1.0;  // both evaluated: no divergent branch\n"
    "  const double e = u < 1.1 ? em1_small : em1_big;\n"
    "  const double t = e / (e + 2.0);\n"
    "  return x == x ? __builtin_copysign(t, x) : x;\n"
    "}\n";

constexpr int64_t kMaxInlineMath = 1024;

std::string math_wrappers(bool f32, const Graph& g, bool inline_math) {
  // T-typed wrappers, plus float ones ("f" suffix) for binary32-tagged
  // instructions of an f64 program.  The inline helpers are emitted only
  // for the operations the program has (other programs' sources, and so
  // their cached code, stay as they are).
  bool has[XG_OP_COUNT] = {false};
  bool has_f32_trig = false;  // binary32-tagged SIN/COS in an f64 program
  int64_t n_inl = 0;
  for (const Node& nd : g.nodes) {
    has[nd.op] = true;
    has_f32_trig = has_f32_trig || (nd.f32 && (nd.op == XG_OP_SIN || nd.op == XG_OP_COS));
    n_inl += nd.op == XG_OP_SIN || nd.op == XG_OP_COS || nd.op == XG_OP_EXP || nd.op == XG_OP_TANH;
  }
  // each inline evaluation is 25-60 instructions: programs with thousands
  // of them would multiply code size and hiprtc time (measured: a 1e4-op
  // random DAG with 4,600 of them, 40 s -> 26 min), so they keep the calls
  if (n_inl > kMaxInlineMath) inline_math = false;
  const bool trig = inline_math && (has[XG_OP_SIN] || has[XG_OP_COS]);
  const bool ex = inline_math && (has[XG_OP_EXP] || has[XG_OP_TANH]);
  const bool th = inline_math && has[XG_OP_TANH];
  auto inlined = [&](int op) {
    return ((op == XG_OP_SIN || op == XG_OP_COS) && trig) || (op == XG_OP_EXP && ex) ||
           (op == XG_OP_TANH && th);
  };
  std::string s;
  if (trig) s += kTrig;
  if (trig && (f32 || has_f32_trig)) s += kTrigF;
  if (ex) s += kExp;
  if (th) s += kTanh;
  for (int pass = 0; pass < (f32 ? 1 : 2); ++pass) {
    const bool fl = f32 || pass == 1;
    const char* ty = pass == 1 ? "float" : "T";
    const char* sfx = pass == 1 ? "f" : "";
    const std::pair<int, const char*> helpers[] = {
        {XG_OP_SIN, "xg_sin_d"}, {XG_OP_COS, "xg_cos_d"}, {XG_OP_EXP, "xg_exp_d"}, {XG_OP_TANH, "xg_tanh_d"}};
    for (auto& h : helpers) {
      if (!inlined(h.first)) continue;
      if (fl && (f32 || has_f32_trig) && (h.first == XG_OP_SIN || h.first == XG_OP_COS))  // binary32 polynomials
        s += std::string("__device__ __forceinline__ ") + ty + " xg_" + op_name(h.first) + sfx + "(" + ty +
             " a) { return " + (h.first == XG_OP_SIN ? "xg_sin_f" : "xg_cos_f") + "(a); }\n";
      else
        s += std::string("__device__ __forceinline__ ") + ty + " xg_" + op_name(h.first) + sfx + "(" + ty +
             " a) { return (" + ty + ")" + h.second + "((double)a); }\n";
    }
    for (int op : {XG_OP_EXP, XG_OP_LOG, XG_OP_SIN, XG_OP_COS, XG_OP_TAN, XG_OP_TANH, XG_OP_ATAN}) {
      if (inlined(op)) continue;
      s += std::string("__device__ __attribute__((noinline)) ") + ty + " xg_" + op_name(op) + sfx +
           "(" + ty + " a) { return " + fn(op, fl) + "(a); }\n";
    }
    for (int op : {XG_OP_POW, XG_OP_ATAN2})
      s += std::string("__device__ __attribute__((noinline)) ") + ty + " xg_" + op_name(op) + sfx +
           "(" + ty + " a, " + ty + " b) { return " + fn(op, fl) + "(a, b); }\n";
  }
  return s;
}

std::string expr(int op, const std::string& A, const std::string& B, const char* ty) {
  switch (op) {
    case XG_OP_ADD: return A + " + " + B;
    case XG_OP_SUB: return A + " - " + B;
    case XG_OP_MUL: return A + " * " + B;
    case XG_OP_DIV: return A + " / " + B;
    case XG_OP_NEG: return "-" + A;
    case XG_OP_SQ: return A + " * " + A;
    case XG_OP_ASSIGN: return A;
    case XG_OP_LT: return "(" + A + " < " + B + " ? " + ty + "(1) : " + ty + "(0))";
    case XG_OP_LE: return "(" + A + " <= " + B + " ? " + ty + "(1) : " + ty + "(0))";
  }
  return std::string();
}

struct ChunkEmitter {
  const Graph& g;
  const Plan& pl;
  const EmitOptions& eo;
  int c;
  bool f32;
  int ipt;
  int R;            // register budget in values (per instance)
  int lds_cap;      // LDS slots per lane available
  int32_t extra_base;
  std::string out;  // body
  EmitStats st;

  // per node state (indexed by node id)
  std::vector<int32_t> chunk_def;      // chunk where the node is scheduled
  std::vector<std::vector<int32_t>> uses;  // use positions in this chunk
  std::vector<int32_t> uptr;
  std::vector<int32_t> nver;           // materialisation counter
  std::vector<int8_t> inreg, loaded, defined;
  std::vector<int32_t> lds_slot, xws_slot;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> outs_of;  // node -> (arg, e)
  int32_t nreg = 0;
  std::priority_queue<std::pair<int32_t, int32_t>> heap;  // (next use, node)
  std::vector<int32_t> lds_free, xws_free;
  int32_t lds_next = 0, xws_next = 0;
  int32_t cur_phase = 0;  // phased plans: barriers emitted so far
  int64_t lds_hi = -1, xch_hi = -1;  // largest LDS byte offsets used (-1: none)

  ChunkEmitter(const Graph& g_, const Plan& pl_, const EmitOptions& eo_, int c_, int32_t xb)
      : g(g_), pl(pl_), eo(eo_), c(c_), extra_base(xb) {
    f32 = g.dtype == XG_F32;
    ipt = std::max(1, eo.ipt);
    R = std::max(4, eo.reg_budget / ipt);
    lds_cap = std::max(0, eo.lds_slots / ipt);
  }

  int32_t nextuse(int32_t v) const {
    return uptr[v] < (int32_t)uses[v].size() ? uses[v][uptr[v]] : kInf;
  }

  std::string name(int32_t v, int r) const {
    std::string s = "v" + std::to_string(v);
    if (nver[v] > 0) s += "_" + std::to_string(nver[v]);
    if (ipt > 1) s += "r" + std::to_string(r);
    return s;
  }

  // C type of a value: float for binary32-tagged nodes, else T
  const char* ctype(int32_t v) const { return g.nodes[v].f32 ? "float" : "T"; }

  // operand v as used by an operation computed in binary32 (as_f32) or in T
  std::string operand(int32_t v, int r, bool as_f32 = false) const {
    const Node& nd = g.nodes[v];
    if (nd.op == XG_OP_CONST) return literal(g.consts[nd.aux], f32 || as_f32);
    const bool vf = nd.f32 || f32;
    const bool want = as_f32 || f32;
    if (vf == want) return name(v, r);
    return std::string(want ? "(float)" : "(T)") + name(v, r);
  }

  // LDS operands "base, offset": the byte offset of (slot, sub-instance r)
  // in this lane's spill region, split into one of the 64 KiB bases the
  // body defines (xg_lb0, xg_lb1, ...) and the 16-bit offset every LDS
  // instruction carries
  std::string lds_at(int32_t slot, int r) {
    const int64_t off = (int64_t)(slot * ipt + r) * eo.block * (f32 ? 4 : 8);
    lds_hi = std::max(lds_hi, off);
    return "xg_lb" + std::to_string(off >> 16) + ", " + std::to_string(off & 0xffff) + "u";
  }
  // workspace element (slot, sub-instance r) of this lane: the block's
  // region is [slot][ipt][block]; slot offsets are compile-time constants
  std::string ws_off(int32_t slot, int r) const {
    return std::to_string((int64_t)(slot * ipt + r) * eo.block * (f32 ? 4 : 8)) + "u";
  }
  std::string wld(int32_t slot, int r) const { return "xg_wld(wsr, " + ws_off(slot, r) + ", tidb)"; }
  std::string wst(int32_t slot, int r, const std::string& v) const {
    return "xg_wst(wsr, " + ws_off(slot, r) + ", tidb, " + v + ");";
  }
  std::string gld(const std::string& base, const std::string& ld, int64_t e, int r) const {
    return "xg_ld(" + base + ", " + ld + ", " + std::to_string(e) + ", ixb" + std::to_string(r) + ")";
  }
  std::string gst(const std::string& base, const std::string& ld, int64_t e, int r,
                  const std::string& val) const {
    return "xg_st(" + base + ", " + ld + ", " + std::to_string(e) + ", ixb" + std::to_string(r) +
           ", " + val + ");";
  }

  void line(const std::string& s) {
    out += "  ";
    out += s;
    out += "\n";
  }
  void guarded(int r, const std::string& s) {
    // Sub-instance 0 stores unconditionally: either lanes past n returned
    // at entry, or (phased plans, where every wave must reach every
    // barrier) their index was clamped to n - 1, so they computed exactly
    // what the lane of instance n - 1 computed and store the same bits to
    // the same place.  A branch per store would cut the straight-line code
    // into many blocks, and the register allocator then spills to scratch.
    if (ipt == 1 || r == 0) line(s);
    else line("if (ok" + std::to_string(r) + ") " + s);
  }
  // phased plans: another wave's value is read from its LDS exchange slot
  // once (the slot is reused after every reader's first read); from then on
  // this wave keeps its own copy like a value it computed
  bool xch_home(int32_t v) const {
    return pl.phased && pl.xch_slot[v] >= 0 && chunk_def[v] != c && !loaded[v];
  }
  // a workspace slot is a value's lasting home except for phased plans,
  // where it is only a one-barrier exchange slot
  bool ws_home(int32_t v) const { return pl.ws_slot[v] >= 0 && !pl.phased; }
  std::string xch_at(int32_t v) {  // as lds_at, in the exchange area (xg_xb0, ...)
    const int64_t off = (int64_t)pl.xch_slot[v] * 64 * (f32 ? 4 : 8);
    xch_hi = std::max(xch_hi, off);
    return "xg_xb" + std::to_string(off >> 16) + ", " + std::to_string(off & 0xffff) + "u";
  }

  bool own(int32_t v) const {  // computed in this chunk (needs a spill slot to leave regs)
    // (phased plans: also another wave's value once read: its exchange slot
    // does not keep it)
    return g.nodes[v].op != XG_OP_INPUT && (chunk_def[v] == c || pl.phased);
  }

  void evict_one(int32_t protect_a, int32_t protect_b) {
    std::vector<std::pair<int32_t, int32_t>> held;
    while (!heap.empty()) {
      auto e = heap.top();
      heap.pop();
      int32_t v = e.second;
      if (!inreg[v] || nextuse(v) != e.first) continue;  // stale
      if (v == protect_a || v == protect_b) { held.push_back(e); continue; }
      // victim v.  A value whose only other copy is in global memory (an
      // input, or a value the workspace holds) also moves to LDS while LDS
      // has room: its reloads then cost LDS latency instead of L2 latency.
      const bool lds_room = !lds_free.empty() || lds_next < lds_cap;
      if (lds_slot[v] < 0 && xws_slot[v] < 0 && lds_room &&
          (!own(v) || ws_home(v))) {
        int32_t s;
        if (!lds_free.empty()) { s = lds_free.back(); lds_free.pop_back(); }
        else s = lds_next++;
        lds_slot[v] = s;
        for (int r = 0; r < ipt; ++r)
          line("xg_lds_st(" + lds_at(s, r) + ", " + name(v, r) + ");");
        st.spills++;
      } else if (own(v) && lds_slot[v] < 0 && xws_slot[v] < 0 && !ws_home(v)) {
        if (lds_room) {
          int32_t s;
          if (!lds_free.empty()) { s = lds_free.back(); lds_free.pop_back(); }
          else s = lds_next++;
          lds_slot[v] = s;
          for (int r = 0; r < ipt; ++r)
            line("xg_lds_st(" + lds_at(s, r) + ", " + name(v, r) + ");");
        } else {
          int32_t s;
          if (!xws_free.empty()) { s = xws_free.back(); xws_free.pop_back(); }
          else s = xws_next++;
          xws_slot[v] = s;
          for (int r = 0; r < ipt; ++r)
            line(wst(extra_base + s, r, name(v, r)));
        }
        st.spills++;
      }
      inreg[v] = 0;
      nreg--;
      break;
    }
    for (auto& e : held) heap.push(e);
  }

  // next use of the value Belady would evict now (kInf if none)
  int32_t farthest_next() {
    while (!heap.empty()) {
      auto e = heap.top();
      if (!inreg[e.second] || nextuse(e.second) != e.first) { heap.pop(); continue; }
      return e.first;
    }
    return kInf;
  }

  void add_reg(int32_t v, int32_t pa, int32_t pb) {
    while (nreg >= R) {
      int before = nreg;
      evict_one(pa, pb);
      if (nreg == before) break;  // nothing evictable
    }
    inreg[v] = 1;
    nreg++;
    heap.push({nextuse(v), v});
  }

  // bring v into registers (new materialisation)
  void materialize(int32_t v, int32_t pa, int32_t pb) {
    const Node& nd = g.nodes[v];
    nver[v]++;
    const bool from_xch = xch_home(v);
    const bool was_loaded = loaded[v] != 0;
    if (lds_slot[v] >= 0 || from_xch || (loaded[v] && nd.op == XG_OP_INPUT)) line("xg_fence();");
    loaded[v] = 1;
    for (int r = 0; r < ipt; ++r) {
      std::string nm = name(v, r);
      if (from_xch) {
        line(std::string("const ") + ctype(v) + " " + nm + " = (" + ctype(v) + ")xg_lds_ld(" + xch_at(v) + ");");
      } else if (lds_slot[v] >= 0) {
        line(std::string("const ") + ctype(v) + " " + nm + " = (" + ctype(v) + ")xg_lds_ld(" + lds_at(lds_slot[v], r) + ");");
      } else if (nd.op == XG_OP_INPUT) {
        int32_t a = (int32_t)(nd.aux >> 32), e = (int32_t)(nd.aux & 0xffffffff);
        line("const T " + nm + " = " + gld("in" + std::to_string(a), "ldi" + std::to_string(a), e, r) + ";");
      } else if (pl.ws_slot[v] >= 0 && (!pl.phased || (chunk_def[v] != c && xws_slot[v] < 0 && !was_loaded))) {
        // crosses a chunk boundary: already in the workspace (phased plans:
        // another wave's value, first read after its phase's barrier)
        line(std::string("const ") + ctype(v) + " " + nm + " = (" + ctype(v) + ")" + wld(pl.ws_slot[v], r) + ";");
      } else {
        line(std::string("const ") + ctype(v) + " " + nm + " = (" + ctype(v) + ")" +
             wld(extra_base + xws_slot[v], r) + ";");
      }
    }
    add_reg(v, pa, pb);
  }

  void release(int32_t v) {  // after its last use in this chunk
    if (inreg[v]) { inreg[v] = 0; nreg--; }
    if (lds_slot[v] >= 0) { lds_free.push_back(lds_slot[v]); lds_slot[v] = -1; }
    if (xws_slot[v] >= 0) { xws_free.push_back(xws_slot[v]); xws_slot[v] = -1; }
  }

  // phased plans: barriers up to phase k, each followed by this wave's
  // copies of the values other waves exchanged in the phase before
  void enter_phase(int32_t k) {
    while (cur_phase < k) {
      line("xg_barrier();");
      ++cur_phase;
      const auto& mb = pl.mailbox[(size_t)c * (pl.n_phases + 1) + cur_phase];
      for (int32_t u : mb)
        if (!inreg[u] && nextuse(u) != kInf) materialize(u, -1, -1);
    }
  }

  void store_outputs(int32_t v) {
    for (auto& ae : outs_of[v])
      for (int r = 0; r < ipt; ++r)
        guarded(r, gst("out" + std::to_string(ae.first), "ldo" + std::to_string(ae.first),
                       ae.second, r, operand(v, r)));
  }

  void run() {
    const int32_t n = (int32_t)g.nodes.size();
    chunk_def.assign(n, -1);
    for (int32_t cc = 0; cc < (int32_t)pl.chunks.size(); ++cc)
      for (int32_t p = pl.chunks[cc].begin; p < pl.chunks[cc].end; ++p) chunk_def[pl.order[p]] = cc;
    if (pl.phased)  // a cheap value several waves compute is this wave's own where it computes it
      for (int32_t p = pl.chunks[c].begin; p < pl.chunks[c].end; ++p) chunk_def[pl.order[p]] = c;
    uses.assign(n, {});
    uptr.assign(n, 0);
    nver.assign(n, -1);
    inreg.assign(n, 0);
    loaded.assign(n, 0);
    defined.assign(n, 0);
    lds_slot.assign(n, -1);
    xws_slot.assign(n, -1);
    outs_of.assign(n, {});
    for (int32_t a = 0; a < (int32_t)g.out.size(); ++a)
      for (int32_t e = 0; e < (int32_t)g.out[a].size(); ++e) outs_of[g.out[a][e]].push_back({a, e});
    const Chunk& ch = pl.chunks[c];
    for (int32_t p = ch.begin; p < ch.end; ++p) {
      const Node& nd = g.nodes[pl.order[p]];
      int32_t a = nd.a, b = nd.b;
      if (a >= 0 && g.nodes[a].op != XG_OP_CONST) uses[a].push_back(p);
      if (b >= 0 && b != a && g.nodes[b].op != XG_OP_CONST) uses[b].push_back(p);
    }
    if (c == 0) {  // outputs that are constants
      for (int32_t v = 0; v < n; ++v)
        if (g.nodes[v].op == XG_OP_CONST && !outs_of[v].empty()) store_outputs(v);
    }
    for (int32_t p = ch.begin; p < ch.end; ++p) {
      int32_t v = pl.order[p];
      const Node& nd = g.nodes[v];
      if (pl.phased) enter_phase(pl.pos_phase[p]);
      if (nd.op == XG_OP_INPUT) {
        // an input is (re)loaded on demand; here only if it is an output
        // or used later in this chunk
        bool needed = !outs_of[v].empty() || nextuse(v) != kInf;
        if (needed && !inreg[v]) materialize(v, -1, -1);
        store_outputs(v);
        if (inreg[v] && nextuse(v) == kInf) release(v);
        continue;
      }
      int32_t a = (nd.a >= 0 && g.nodes[nd.a].op != XG_OP_CONST) ? nd.a : -1;
      int32_t b = (nd.b >= 0 && g.nodes[nd.b].op != XG_OP_CONST) ? nd.b : -1;
      // issue now the reloads needed `prefetch` positions ahead (LDS
      // latency) and the global-memory reloads (inputs and workspace values
      // not held in LDS) needed four times as far ahead, so their latency
      // overlaps this stretch of arithmetic
      for (int far = 0; far < 2 && eo.prefetch > 0; ++far) {
        const int32_t dist = far ? 4 * eo.prefetch : eo.prefetch;
        if (p + dist >= ch.end) continue;
        const Node& fn_ = g.nodes[pl.order[p + dist]];
        for (int32_t o : {fn_.a, fn_.b}) {
          if (o < 0 || g.nodes[o].op == XG_OP_CONST || inreg[o]) continue;
          if (g.nodes[o].op != XG_OP_INPUT && chunk_def[o] == c && !defined[o])
            continue;  // not yet computed (defined between here and its use)
          if (pl.phased && chunk_def[o] != c && g.nodes[o].op != XG_OP_INPUT &&
              pl.node_phase[o] >= cur_phase)
            continue;  // another wave's value: readable after its phase's barrier
          if (far && (lds_slot[o] >= 0 || xch_home(o))) continue;  // an LDS reload: the near distance covers it
          if (nreg >= R && farthest_next() <= p + dist) continue;  // would evict sooner uses
          materialize(o, a, b);
        }
      }
      if (a >= 0 && !inreg[a]) materialize(a, a, b);
      if (b >= 0 && b != a && !inreg[b]) materialize(b, a, b);
      nver[v]++;
      defined[v] = 1;
      const bool nf = nd.f32 != 0;  // binary32 instruction in an f64 program
      for (int r = 0; r < ipt; ++r) {
        std::string A = nd.a >= 0 ? operand(nd.a, r, nf) : "";
        std::string B = nd.b >= 0 ? operand(nd.b, r, nf) : "";
        std::string e = expr(nd.op, A, B, ctype(v));
        if (e.empty()) {
          std::string f = (eo.call_math && outlined(nd.op))
                              ? std::string("xg_") + op_name(nd.op) + (nf ? "f" : "")
                              : std::string(fn(nd.op, f32 || nf));
          e = f + "(" + A + (is_binary(nd.op) ? ", " + B : std::string()) + ")";
        }
        line(std::string("const ") + ctype(v) + " " + name(v, r) + " = " + e + ";");
      }
      // operands: advance past this use
      const int32_t b2 = (b == a) ? -1 : b;
      for (int32_t o : {a, b2}) {
        if (o < 0) continue;
        uptr[o]++;
        if (nextuse(o) == kInf) release(o);
        else if (inreg[o]) heap.push({nextuse(o), o});
      }
      store_outputs(v);
      if (pl.ws_slot[v] >= 0)
        for (int r = 0; r < ipt; ++r) line(wst(pl.ws_slot[v], r, name(v, r)));
      if (pl.phased && pl.xch_slot[v] >= 0)
        line("xg_lds_st(" + xch_at(v) + ", " + name(v, 0) + ");");
      if (nextuse(v) != kInf) add_reg(v, a, b);
    }
    if (pl.phased) enter_phase(pl.n_phases - 1);  // every wave passes every barrier
    st.lds_slots = lds_next * ipt;
    st.extra_ws = xws_next;
    // the LDS bases: this lane's address in the region plus k * 64 KiB,
    // each passed through an empty asm so that the compiler keeps it in one
    // register and folds every access's constant into the instruction's
    // offset field (a constant beyond 64 KiB it would otherwise add to the
    // lane offset again for every access)
    std::string bases;
    auto define = [&](const std::string& nm, const char* region, int64_t hi) {
      if (hi < 0) return;
      bases += "  unsigned " + nm + "0 = (unsigned)(size_t)(lC*)" + region + " + tidb;\n";
      bases += "  asm volatile(\"\" : \"+v\"(" + nm + "0));\n";
      for (int64_t k = 1; k <= (hi >> 16); ++k) {
        const std::string K = std::to_string(k);
        bases += "  unsigned " + nm + K + " = " + nm + "0 + " + std::to_string(k * 65536) + "u;\n";
        bases += "  asm volatile(\"\" : \"+v\"(" + nm + K + "));\n";
      }
    };
    define("xg_lb", "lds", lds_hi);
    define("xg_xb", "xch", xch_hi);
    out = bases + out;
  }
};

std::string dtype_name(const Graph& g) { return g.dtype == XG_F32 ? "float" : "double"; }

// Emitted once per source.  A global access forms its address at the
// point of use from a uniform base (kernel argument, SGPRs) that passes
// through an empty asm, plus the lane's 32-bit byte offset: the optimiser
// can then neither merge two accesses' addresses nor hoist them (it would
// otherwise keep one 64-bit address per slot live from the first access to
// the last, costing more registers than the values), and the address maps
// onto the "SGPR base + VGPR offset" global addressing mode with no vector
// instruction spent on it.  xg_fence() is a compiler-only memory barrier
// placed before every reload, so a reload is never replaced by the value of
// the earlier store to the same slot.
const char* kAccessHelpers =
    "typedef __attribute__((address_space(1))) T gT;\n"
    "typedef __attribute__((address_space(1))) char gC;\n"
    "typedef __attribute__((address_space(3))) T lT;\n"
    "typedef __attribute__((address_space(3))) char lC;\n"
    "#define xg_fence() asm volatile(\"\" ::: \"memory\")\n"
    "__device__ __forceinline__ T xg_ld(const T* p, long long ld, long long e, unsigned o) {\n"
    "  const gT* g = (const gT*)p;\n"
    "  asm volatile(\"\" : \"+s\"(g), \"+s\"(ld));\n"
    "  return *(const gT*)((const gC*)(g + e * ld) + o);\n"
    "}\n"
    "__device__ __forceinline__ void xg_st(T* p, long long ld, long long e, unsigned o, T v) {\n"
    "  gT* g = (gT*)p;\n"
    "  asm volatile(\"\" : \"+s\"(g), \"+s\"(ld));\n"
    "  *(gT*)((gC*)(g + e * ld) + o) = v;\n"
    "}\n"
    "__device__ __forceinline__ T xg_lds_ld(unsigned b, unsigned c) {\n"
    "  return *(lT*)(size_t)(b + c);\n"
    "}\n"
    "__device__ __forceinline__ void xg_lds_st(unsigned b, unsigned c, T v) {\n"
    "  *(lT*)(size_t)(b + c) = v;\n"
    "}\n";

std::string index_prologue(const EmitOptions& eo, int ipt, bool clamp = false) {
  std::string s;
  s += eo.waves > 1 ? "  const int tid = threadIdx.x & 63;\n" : "  const int tid = threadIdx.x;\n";
  s += "  const unsigned tidb = (unsigned)tid * (unsigned)sizeof(T);\n";
  for (int r = 0; r < ipt; ++r) {
    std::string R = std::to_string(r);
    s += "  const long long iv" + R + " = ibase + " + std::to_string(r * eo.block) + ";\n";
    if (r == 0 && !clamp) {
      s += "  if (iv0 >= n) return;\n  const long long ix0 = iv0;\n";
    } else {
      s += "  const bool ok" + R + " = iv" + R + " < n;\n";
      s += "  const long long ix" + R + " = ok" + R + " ? iv" + R + " : n - 1;\n";
    }
    s += "  const unsigned ixb" + R + " = (unsigned)ix" + R + " * (unsigned)sizeof(T);\n";
  }
  return s;
}

}  // namespace

std::string ws_prologue(const EmitOptions& eo, int64_t ns, const char* blk) {
  if (ns <= 0) return std::string();
  const int ipt = std::max(1, eo.ipt);
  const std::string per = std::to_string(ns * ipt * eo.block);
  return std::string("  const __amdgpu_buffer_rsrc_t wsr = __builtin_amdgcn_make_buffer_rsrc(") +
         "(void*)(ws + (long long)(" + blk + ") * " + per + "), (short)0, (int)(" + per +
         " * sizeof(T)), 0x00020000);\n";
}

std::vector<std::string> emit_chunks(const Graph& g, const Plan& plan, const EmitOptions& eo,
                                     const std::string& prefix, EmitStats* st,
                                     int32_t extra_ws_base) {
  const int ipt = std::max(1, eo.ipt);
  const int nc = (int)plan.chunks.size();
  std::vector<std::unique_ptr<ChunkEmitter>> ces;
  EmitStats tot;
  for (int c = 0; c < nc; ++c) {
    ces.emplace_back(new ChunkEmitter(g, plan, eo, c, extra_ws_base));
    ces.back()->out.reserve((size_t)(plan.chunks[c].end - plan.chunks[c].begin) * 64 * ipt + 4096);
    ces.back()->run();
    tot.spills += ces.back()->st.spills;
    tot.lds_slots = std::max(tot.lds_slots, ces.back()->st.lds_slots);
    tot.extra_ws = std::max(tot.extra_ws, ces.back()->st.extra_ws);
  }
  const int64_t ns = (int64_t)extra_ws_base + tot.extra_ws;  // workspace slots per instance
  std::vector<std::string> srcs;
  for (int c = 0; c < nc; ++c) {
    ChunkEmitter& ce = *ces[c];
    std::string s;
    s.reserve(ce.out.size() + 4096);
    s += "// generated by xg: chunk " + std::to_string(c) + " of " + std::to_string(nc) + "\n";
    s += contract_pragma(eo.strict);
    s += emit_preamble(g, eo);
    s += "extern \"C\" __global__ void __launch_bounds__(" + std::to_string(eo.block) + ") " +
         prefix + "_c" + std::to_string(c) + "(long long n";
    for (size_t a = 0; a < g.nnz_in.size(); ++a)
      s += ", const T* __restrict__ in" + std::to_string(a) + ", long long ldi" + std::to_string(a);
    for (size_t a = 0; a < g.nnz_out.size(); ++a)
      s += ", T* __restrict__ out" + std::to_string(a) + ", long long ldo" + std::to_string(a);
    s += ", T* __restrict__ ws) {\n";
    s += "  const long long ibase = (long long)blockIdx.x * " + std::to_string(eo.block * ipt) +
         " + threadIdx.x;\n";
    s += index_prologue(eo, ipt);
    s += ws_prologue(eo, ns, "blockIdx.x");
    if (ce.st.lds_slots > 0) {
      s += "  __shared__ T lds_[" + std::to_string((int64_t)ce.st.lds_slots * eo.block) + "];\n";
      s += "  lT* lds = (lT*)lds_;\n";
    }
    s += ce.out;
    s += "}\n";
    srcs.push_back(std::move(s));
  }
  if (st) *st = tot;
  return srcs;
}

// Workspace accesses: raw buffer loads/stores (resource = the block's
// workspace region, SGPRs; offsets = constant slot offset + lane offset).
std::string buffer_helpers(bool f32) {
  const char* bits = f32 ? "32" : "64";
  const char* vt = f32 ? "unsigned" : "xg_u2";
  std::string s = "typedef unsigned int xg_u2 __attribute__((ext_vector_type(2)));\n";
  s += std::string("__device__ __forceinline__ T xg_wld(__amdgpu_buffer_rsrc_t r, unsigned so, unsigned vo) {\n") +
       "  return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b" + bits + "(r, vo, so, 0));\n}\n";
  s += std::string("__device__ __forceinline__ void xg_wst(__amdgpu_buffer_rsrc_t r, unsigned so, unsigned vo, T v) {\n") +
       "  __builtin_amdgcn_raw_buffer_store_b" + bits + "(__builtin_bit_cast(" + vt + ", v), r, vo, so, 0);\n}\n";
  return s;
}

// Outside strict mode the generated code lets the compiler fuse a multiply
// and a dependent add across statements into one FMA.  The permission is
// given by this pragma (per instruction) with -ffp-contract=on, not by
// -ffp-contract=fast: the latter is a code-generator setting that also fuses
// inside linked device-library functions, whose error-free transformations
// rely on separate roundings (pow lost up to 26 ulp that way).
std::string contract_pragma(bool strict) {
  return strict ? std::string() : std::string("#pragma clang fp contract(fast)\n");
}

std::string emit_preamble(const Graph& g, const EmitOptions& eo) {
  std::string s = "typedef " + dtype_name(g) + " T;\n";
  s += kAccessHelpers;
  s += buffer_helpers(g.dtype == XG_F32);
  if (eo.call_math) s += math_wrappers(g.dtype == XG_F32, g, eo.inline_math);
  return s;
}

WideParts emit_wide_parts(const Graph& g, const Plan& plan, const EmitOptions& eo,
                          const std::string& args_prologue, const std::string& lds_array,
                          const std::string& fprefix) {
  const int nc = (int)plan.chunks.size();
  WideParts wp;
  // pass 1: every chunk's own global spill need (chunks of one phase run
  // concurrently, so each gets a private range of extra workspace slots)
  std::vector<int32_t> xbase(nc + 1, plan.n_ws);
  int32_t lds_need = 0;
  for (int c = 0; c < nc; ++c) {
    ChunkEmitter ce(g, plan, eo, c, 0);
    if (plan.chunks[c].end > plan.chunks[c].begin || c == 0) ce.run();
    xbase[c + 1] = xbase[c] + ce.st.extra_ws;
    lds_need = std::max(lds_need, ce.st.lds_slots);
  }
  wp.ns = xbase[nc];
  wp.lds_wave_elems = (int64_t)lds_need * 64;
  std::string pro = args_prologue;
  if (wp.lds_wave_elems > 0)
    pro += "  lT* lds = (lT*)" + lds_array + " + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * " +
           std::to_string(wp.lds_wave_elems) + ";\n";
  // pass 2: chunk bodies with their final extra-slot bases
  std::vector<char> has_code(nc, 0);
  for (int c = 0; c < nc; ++c) {
    if (!(plan.chunks[c].end > plan.chunks[c].begin || c == 0)) continue;
    ChunkEmitter ce(g, plan, eo, c, xbase[c]);
    ce.run();
    if (ce.out.empty()) continue;
    has_code[c] = 1;
    wp.st.spills += ce.st.spills;
    wp.st.lds_slots = std::max(wp.st.lds_slots, ce.st.lds_slots);
    wp.funcs += "__device__ __attribute__((noinline)) void " + fprefix + std::to_string(c) + "(long long ibase) {\n";
    wp.funcs += pro;
    wp.funcs += index_prologue(eo, 1);
    wp.funcs += "  const int xg_tile = __builtin_amdgcn_readfirstlane((int)(ibase >> 6));\n";
    wp.funcs += ws_prologue(eo, wp.ns, "xg_tile");
    wp.funcs += ce.out;
    wp.funcs += "}\n";
  }
  wp.st.extra_ws = (int32_t)(wp.ns - plan.n_ws);
  // phase sequence, run by every wave of the workgroup with the wave index
  // xg_w and the lane's instance ibase in scope; a barrier separates two
  // phases that both run code (the workspace values one phase stores are
  // read by later phases on other waves)
  int c = 0;
  bool pending = false;  // code ran since the last barrier
  for (int ph = 0; ph < plan.n_phases; ++ph) {
    std::string calls;
    bool first = true;
    for (; c < nc && plan.chunk_phase[c] == ph; ++c) {
      if (!has_code[c]) continue;
      calls += std::string(first ? "  if" : "  else if") + " (xg_w == " + std::to_string(plan.chunk_wave[c]) +
               ") " + fprefix + std::to_string(c) + "(ibase);\n";
      first = false;
    }
    if (calls.empty()) continue;
    if (pending) wp.body += "  __syncthreads();\n";
    wp.body += calls;
    pending = true;
  }
  return wp;
}

std::vector<std::string> emit_wide(const Graph& g, const Plan& plan, const EmitOptions& eo,
                                   const std::string& prefix, EmitStats* st) {
  const int W = plan.waves;
  std::string args = "struct XgArgs { long long n;";
  for (size_t a = 0; a < g.nnz_in.size(); ++a)
    args += " const T* in" + std::to_string(a) + "; long long ldi" + std::to_string(a) + ";";
  for (size_t a = 0; a < g.nnz_out.size(); ++a)
    args += " T* out" + std::to_string(a) + "; long long ldo" + std::to_string(a) + ";";
  args += " T* ws; };\n";
  std::string pro = "  const XgArgs& A = *XG_ARGS;\n  const long long n = A.n; T* __restrict__ ws = A.ws;\n";
  for (size_t a = 0; a < g.nnz_in.size(); ++a)
    pro += "  const T* __restrict__ in" + std::to_string(a) + " = A.in" + std::to_string(a) +
           "; const long long ldi" + std::to_string(a) + " = A.ldi" + std::to_string(a) + ";\n";
  for (size_t a = 0; a < g.nnz_out.size(); ++a)
    pro += "  T* __restrict__ out" + std::to_string(a) + " = A.out" + std::to_string(a) +
           "; const long long ldo" + std::to_string(a) + " = A.ldo" + std::to_string(a) + ";\n";
  WideParts wp = emit_wide_parts(g, plan, eo, pro, "xg_lds_raw", "xg_g");
  std::string s;
  s += "// generated by xg: cooperative tile of " + std::to_string(W) + " waves, " +
       std::to_string(plan.n_phases) + " phases, " + std::to_string(plan.chunks.size()) + " chunks\n";
  s += contract_pragma(eo.strict);
  s += emit_preamble(g, eo);
  s += args;
  // kernel arguments are 8-byte values laid out back to back, as in XgArgs;
  // the implicit arguments follow them (checked on the host against the
  // code object's metadata before the kernel is loaded)
  s += "#define XG_ARGS ((const XgArgs*)((const char*)__builtin_amdgcn_implicitarg_ptr() - sizeof(XgArgs)))\n";
  if (wp.lds_wave_elems > 0)
    s += "__shared__ __attribute__((aligned(16))) T xg_lds_raw[" + std::to_string(wp.lds_wave_elems * W) + "];\n";
  s += wp.funcs;
  s += "extern \"C\" __global__ void __launch_bounds__(" + std::to_string(64 * W) + ") " + prefix +
       "_c0(long long n";
  for (size_t a = 0; a < g.nnz_in.size(); ++a)
    s += ", const T* __restrict__ in" + std::to_string(a) + ", long long ldi" + std::to_string(a);
  for (size_t a = 0; a < g.nnz_out.size(); ++a)
    s += ", T* __restrict__ out" + std::to_string(a) + ", long long ldo" + std::to_string(a);
  s += ", T* __restrict__ ws) {\n";
  s += "  const int xg_w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));\n";
  s += "  const long long ibase = (long long)blockIdx.x * 64 + (threadIdx.x & 63);\n";
  s += wp.body;
  s += "}\n";
  if (st) *st = wp.st;
  return {s};
}

namespace {

// The waves' code of a phased plan: an if / else-if chain on xg_w, one
// branch per wave holding its straight-line share with the phase barriers
// inline.  Also returns the workspace slots per instance (the plan's, then
// each wave's private range for its own spills, as the waves run at once)
// and the LDS elements of one wave's spill region.
struct PhasedBranches {
  std::string code;
  int64_t ns = 0;
  int64_t lds_wave_elems = 0;
  EmitStats st;
};

PhasedBranches phased_branches(const Graph& g, const Plan& plan, const EmitOptions& eo_in) {
  const int W = plan.waves;
  const int64_t es = g.dtype == XG_F32 ? 4 : 8;
  // LDS: the exchange slots, then one spill region per wave in what is left
  EmitOptions eo = eo_in;
  const int64_t xch_bytes = (int64_t)plan.n_xch * 64 * es;
  const int64_t spill_cap = std::max<int64_t>(0, (160 * 1024 - 512 - xch_bytes) / (64 * W * es));
  eo.lds_slots = (int)std::min<int64_t>(eo.lds_slots, spill_cap);
  // pass 1: each wave's own global spill need
  std::vector<int32_t> xbase(W + 1, plan.n_ws);
  int32_t lds_need = 0;
  for (int c = 0; c < W; ++c) {
    ChunkEmitter ce(g, plan, eo, c, 0);
    ce.run();
    xbase[c + 1] = xbase[c] + ce.st.extra_ws;
    lds_need = std::max(lds_need, ce.st.lds_slots);
  }
  PhasedBranches pb;
  pb.ns = xbase[W];
  pb.lds_wave_elems = (int64_t)lds_need * 64;
  for (int c = 0; c < W; ++c) {
    ChunkEmitter ce(g, plan, eo, c, xbase[c]);
    ce.run();
    pb.st.spills += ce.st.spills;
    pb.st.lds_slots = std::max(pb.st.lds_slots, ce.st.lds_slots);
    pb.code += std::string(c == 0 ? "  if" : "  else if") + " (xg_w == " + std::to_string(c) + ") {\n";
    pb.code += ce.out;
    pb.code += "  }\n";
  }
  pb.st.extra_ws = (int32_t)(pb.ns - plan.n_ws);
  return pb;
}

}  // namespace

std::vector<std::string> emit_phased(const Graph& g, const Plan& plan, const EmitOptions& eo,
                                     const std::string& prefix, EmitStats* st) {
  const int W = plan.waves;
  PhasedBranches pb = phased_branches(g, plan, eo);
  std::string s;
  s += "// generated by xg: phased cooperative tile of " + std::to_string(W) + " waves, " +
       std::to_string(plan.n_phases) + " phases, " + std::to_string(plan.n_xch) + " exchange slots\n";
  s += contract_pragma(eo.strict);
  s += emit_preamble(g, eo);
  s += "#define xg_barrier() __syncthreads()\n";
  s += "extern \"C\" __global__ void __launch_bounds__(" + std::to_string(64 * W) + ") " + prefix +
       "_c0(long long n";
  for (size_t a = 0; a < g.nnz_in.size(); ++a)
    s += ", const T* __restrict__ in" + std::to_string(a) + ", long long ldi" + std::to_string(a);
  for (size_t a = 0; a < g.nnz_out.size(); ++a)
    s += ", T* __restrict__ out" + std::to_string(a) + ", long long ldo" + std::to_string(a);
  s += ", T* __restrict__ ws) {\n";
  // the wave index is uniform (readfirstlane): each branch below is taken
  // by whole waves, and every branch passes the same number of barriers
  s += "  const int xg_w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));\n";
  s += "  const long long ibase = (long long)blockIdx.x * 64 + (threadIdx.x & 63);\n";
  s += index_prologue(eo, 1, true);
  s += "  const int xg_tile = blockIdx.x;\n";
  s += ws_prologue(eo, pb.ns, "xg_tile");
  if (pb.lds_wave_elems > 0) {
    s += "  __shared__ __attribute__((aligned(16))) T xg_lds_raw[" + std::to_string(pb.lds_wave_elems * W) + "];\n";
    s += "  lT* lds = (lT*)xg_lds_raw + xg_w * " + std::to_string(pb.lds_wave_elems) + ";\n";
  }
  if (plan.n_xch > 0) {
    s += "  __shared__ __attribute__((aligned(16))) T xg_xch_raw[" + std::to_string((int64_t)plan.n_xch * 64) + "];\n";
    s += "  lT* xch = (lT*)xg_xch_raw;\n";
  }
  s += pb.code;
  s += "}\n";
  if (st) *st = pb.st;
  return {s};
}

PhasedParts emit_phased_parts(const Graph& g, const Plan& plan, const EmitOptions& eo,
                              const std::string& lds_array) {
  const int W = plan.waves;
  const int64_t es = g.dtype == XG_F32 ? 4 : 8;
  PhasedBranches pb = phased_branches(g, plan, eo);
  PhasedParts pp;
  pp.ns = pb.ns;
  pp.st = pb.st;
  const int64_t xch_elems = (int64_t)plan.n_xch * 64;
  pp.lds_bytes = (xch_elems + pb.lds_wave_elems * W) * es;
  std::string& s = pp.body;
  s += index_prologue(eo, 1, true);
  // the lanes of a wave share one tile: ibase / 64 is uniform
  s += "  const int xg_tile = __builtin_amdgcn_readfirstlane((int)(ibase >> 6));\n";
  s += ws_prologue(eo, pb.ns, "xg_tile");
  // one LDS array: the exchange slots first, then the waves' spill regions
  if (plan.n_xch > 0) s += "  lT* xch = (lT*)" + lds_array + ";\n";
  if (pb.lds_wave_elems > 0)
    s += "  lT* lds = (lT*)" + lds_array + " + " + std::to_string(xch_elems) + " + xg_w * " +
         std::to_string(pb.lds_wave_elems) + ";\n";
  s += pb.code;
  return pp;
}

std::string emit_device_chunk(const Graph& g, const Plan& plan, int c, const EmitOptions& eo,
                              const std::string& fname, const std::string& prologue,
                              EmitStats* st, int32_t extra_ws_base, int64_t ns) {
  const int ipt = std::max(1, eo.ipt);
  ChunkEmitter ce(g, plan, eo, c, extra_ws_base);
  ce.run();
  std::string s;
  s.reserve(ce.out.size() + 2048);
  s += "__device__ __attribute__((noinline)) void " + fname + "(long long ibase) {\n";
  s += prologue;
  s += index_prologue(eo, ipt);
  s += "  const int xg_tile = __builtin_amdgcn_readfirstlane((int)(ibase / " +
       std::to_string(eo.block * ipt) + "));\n";
  s += ws_prologue(eo, ns, "xg_tile");
  s += ce.out;
  s += "}\n";
  if (st) *st = ce.st;
  return s;
}

}  // namespace xg
