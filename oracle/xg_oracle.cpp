// Oracle: a plain sequential interpreter of work-vector programs.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file's library; only the tests, the smoke check and the
// benchmark's CPU-baseline leg use it.  It shares no code with the GPU
// library (own parser, own opcode table, own semantics).
//
// What it computes.  The paper's "Code Generation" section defines the
// function as a work vector plus a list of instructions (operation id,
// operand indices, output index), evaluated by traversing the instructions
// in order and applying each operation to the indexed entries.  The GPU
// method reaches exactly that result (each instruction becomes one
// statement of the generated kernel, run by one thread per instance), so
// the oracle IS that definition: for every instance, independently, walk
// the instructions in order; every instruction reads all of its operands
// before it writes its output slot (the generated-kernel listing writes
// slot 1 from slot 1).  INPUT reads element `nz` of input argument `arg`;
// OUTPUT writes element `nz` of output argument `arg`.  Inputs and outputs
// are the dense vectors of structural non-zeros (background section on
// sparsity: only non-zeros are computed and passed).
//
// Scalar types: float, double, long double (x87 80-bit) and a dual number
// over double carrying K tangent directions (forward-mode derivatives, the
// exact derivative up to rounding).  Compiled with -O2 -ffp-contract=off
// and without -ffast-math: no contraction, round-to-nearest-even,
// denormals kept.
//
// Parity status of each part is stated in the oracle README.

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

namespace {

enum Op {
  O_INPUT, O_OUTPUT, O_CONST, O_ASSIGN,
  O_ADD, O_SUB, O_MUL, O_DIV,
  O_NEG, O_SQ, O_SQRT, O_EXP, O_LOG,
  O_SIN, O_COS, O_TAN, O_TANH, O_ATAN,
  O_FABS, O_FMIN, O_FMAX, O_LT, O_LE,
  O_POW, O_ATAN2,
  O_COUNT
};

const char* kOpNames[O_COUNT] = {
  "INPUT", "OUTPUT", "CONST", "ASSIGN",
  "ADD", "SUB", "MUL", "DIV",
  "NEG", "SQ", "SQRT", "EXP", "LOG",
  "SIN", "COS", "TAN", "TANH", "ATAN",
  "FABS", "FMIN", "FMAX", "LT", "LE",
  "POW", "ATAN2",
};

bool binary(int op) {
  return op == O_ADD || op == O_SUB || op == O_MUL || op == O_DIV || op == O_FMIN ||
         op == O_FMAX || op == O_LT || op == O_LE || op == O_POW || op == O_ATAN2;
}

struct Instr { int op; long long out, a, b; bool f32 = false; };

struct Prog {
  std::string name, dtype;
  long long n_work = 0;
  std::vector<long long> nnz_in, nnz_out;
  std::vector<double> consts;
  std::vector<Instr> ins;
  long long tot_in = 0, tot_out = 0;
  std::vector<long long> off_in, off_out;  // prefix offsets of args
};

// ---------------------------------------------------------------- parser
bool parse(const char* path, Prog& p, std::string& err) {
  std::ifstream f(path);
  if (!f) { err = std::string("cannot open ") + path; return false; }
  std::string key;
  long long ver = 0;
  if (!(f >> key >> ver) || key != "xgprog" || ver != 1) { err = "bad header"; return false; }
  auto expect = [&](const char* k) {
    std::string s;
    if (!(f >> s) || s != k) { err = std::string("expected ") + k; return false; }
    return true;
  };
  if (!expect("name") || !(f >> p.name)) return false;
  if (!expect("dtype") || !(f >> p.dtype)) return false;
  if (!expect("n_work") || !(f >> p.n_work)) return false;
  long long k = 0;
  if (!expect("inputs") || !(f >> k) || k < 0) { err = "bad inputs"; return false; }
  p.nnz_in.resize(k);
  for (auto& v : p.nnz_in) if (!(f >> v) || v < 0) { err = "bad nnz_in"; return false; }
  if (!expect("outputs") || !(f >> k) || k < 0) { err = "bad outputs"; return false; }
  p.nnz_out.resize(k);
  for (auto& v : p.nnz_out) if (!(f >> v) || v < 0) { err = "bad nnz_out"; return false; }
  if (!expect("consts") || !(f >> k) || k < 0) { err = "bad consts"; return false; }
  p.consts.resize(k);
  for (auto& c : p.consts) {
    std::string s;
    if (!(f >> s)) { err = "bad const"; return false; }
    char* end = nullptr;
    c = std::strtod(s.c_str(), &end);  // accepts C99 hex floats exactly
    if (end == s.c_str() || *end) { err = "bad const " + s; return false; }
  }
  if (!expect("instrs") || !(f >> k) || k < 0) { err = "bad instrs"; return false; }
  p.ins.resize(k);
  for (long long i = 0; i < k; ++i) {
    std::string name;
    Instr& in = p.ins[i];
    if (!(f >> name >> in.out >> in.a >> in.b)) { err = "bad instr " + std::to_string(i); return false; }
    in.op = -1;
    for (int o = 0; o < O_COUNT; ++o) if (name == kOpNames[o]) in.op = o;
    if (in.op < 0) { err = "unknown op " + name + " at " + std::to_string(i); return false; }
  }
  // optional: instructions computed in binary32 inside an f64 program
  std::string tok;
  if (!(f >> tok)) { err = "expected end"; return false; }
  if (tok == "prec") {
    long long np = 0;
    if (!(f >> np) || np < 0) { err = "bad prec"; return false; }
    for (long long j = 0; j < np; ++j) {
      long long idx;
      std::string v;
      if (!(f >> idx >> v) || idx < 0 || idx >= k || v != "f32") { err = "bad prec entry"; return false; }
      p.ins[idx].f32 = true;
    }
    if (!(f >> tok)) { err = "expected end"; return false; }
  }
  if (tok != "end") { err = "expected end"; return false; }
  p.off_in.assign(p.nnz_in.size() + 1, 0);
  for (size_t a = 0; a < p.nnz_in.size(); ++a) p.off_in[a + 1] = p.off_in[a] + p.nnz_in[a];
  p.off_out.assign(p.nnz_out.size() + 1, 0);
  for (size_t a = 0; a < p.nnz_out.size(); ++a) p.off_out[a + 1] = p.off_out[a] + p.nnz_out[a];
  p.tot_in = p.off_in.back();
  p.tot_out = p.off_out.back();
  return true;
}

// Reject anything whose meaning is not defined: out-of-range indices, a
// read of a slot never written, an output element never written.
bool validate(const Prog& p, std::string& err) {
  std::vector<char> written(p.n_work, 0);
  std::vector<std::vector<char>> outw(p.nnz_out.size());
  for (size_t a = 0; a < p.nnz_out.size(); ++a) outw[a].assign(p.nnz_out[a], 0);
  auto slot_ok = [&](long long s) { return s >= 0 && s < p.n_work; };
  for (size_t i = 0; i < p.ins.size(); ++i) {
    const Instr& in = p.ins[i];
    std::string at = " at instruction " + std::to_string(i);
    auto rd = [&](long long s) {
      if (!slot_ok(s)) { err = "slot out of range" + at; return false; }
      if (!written[s]) { err = "read before write" + at; return false; }
      return true;
    };
    switch (in.op) {
      case O_INPUT:
        if (in.a < 0 || in.a >= (long long)p.nnz_in.size() || in.b < 0 || in.b >= p.nnz_in[in.a]) {
          err = "input index out of range" + at; return false;
        }
        break;
      case O_CONST:
        if (in.a < 0 || in.a >= (long long)p.consts.size()) { err = "const index out of range" + at; return false; }
        break;
      case O_OUTPUT:
        if (in.out < 0 || in.out >= (long long)p.nnz_out.size() || in.b < 0 || in.b >= p.nnz_out[in.out]) {
          err = "output index out of range" + at; return false;
        }
        if (!rd(in.a)) return false;
        outw[in.out][in.b] = 1;
        continue;
      default:
        if (!rd(in.a)) return false;
        if (binary(in.op) && !rd(in.b)) return false;
    }
    if (in.f32 && (p.dtype != "f64" || in.op == O_INPUT || in.op == O_CONST)) {
      err = "f32 tag only on arithmetic of an f64 program" + at; return false;
    }
    if (!slot_ok(in.out)) { err = "slot out of range" + at; return false; }
    written[in.out] = 1;
  }
  for (size_t a = 0; a < outw.size(); ++a)
    for (size_t e = 0; e < outw[a].size(); ++e)
      if (!outw[a][e]) { err = "output " + std::to_string(a) + "[" + std::to_string(e) + "] never written"; return false; }
  return true;
}

// ------------------------------------------------------- scalar semantics
// Plain types: the C99 / C++ library functions (the float overloads call
// the single-precision routines, the long double ones the x87 routines).
template <class S> S s_const(double c) { return (S)c; }
template <class S> S s_sq(S a) { return a * a; }
template <class S> S s_lt(S a, S b) { return a < b ? S(1) : S(0); }
template <class S> S s_le(S a, S b) { return a <= b ? S(1) : S(0); }

template <class S>
S apply(int op, S a, S b) {
  switch (op) {
    case O_ADD: return a + b;
    case O_SUB: return a - b;
    case O_MUL: return a * b;
    case O_DIV: return a / b;
    case O_NEG: return -a;
    case O_SQ: return s_sq(a);
    case O_SQRT: return std::sqrt(a);
    case O_EXP: return std::exp(a);
    case O_LOG: return std::log(a);
    case O_SIN: return std::sin(a);
    case O_COS: return std::cos(a);
    case O_TAN: return std::tan(a);
    case O_TANH: return std::tanh(a);
    case O_ATAN: return std::atan(a);
    case O_FABS: return std::fabs(a);
    case O_FMIN: return std::fmin(a, b);
    case O_FMAX: return std::fmax(a, b);
    case O_LT: return s_lt(a, b);
    case O_LE: return s_le(a, b);
    case O_POW: return std::pow(a, b);
    case O_ATAN2: return std::atan2(a, b);
    case O_ASSIGN: return a;
  }
  std::abort();
}

// Dual number: value v and K tangents in scalar type S (double: v is
// bitwise the double interpreter's value; float: every value and tangent
// operation in binary32), propagated by the chain rule of each opcode.  Tie
// rules: FMIN/FMAX send the derivative to the first operand on a tie;
// FABS'(0) = 0; comparisons have zero derivative.
template <class S>
struct Dual {
  S v;
  std::vector<S> d;
};

template <class S>
void dual_apply(int op, const Dual<S>& a, const Dual<S>& b, Dual<S>& r, int K) {
  const S va = a.v, vb = b.v;
  const S v = apply<S>(op, va, vb);
  const S one = S(1), zero = S(0);
  S da = zero, db = zero;  // partial derivatives w.r.t. a and b
  bool use_b = binary(op);
  switch (op) {
    case O_ADD: da = one; db = one; break;
    case O_SUB: da = one; db = -one; break;
    case O_MUL: da = vb; db = va; break;
    case O_DIV: da = one / vb; db = -va / (vb * vb); break;
    case O_NEG: da = -one; break;
    case O_ASSIGN: da = one; break;
    case O_SQ: da = S(2) * va; break;
    case O_SQRT: da = one / (S(2) * v); break;
    case O_EXP: da = v; break;
    case O_LOG: da = one / va; break;
    case O_SIN: da = std::cos(va); break;
    case O_COS: da = -std::sin(va); break;
    case O_TAN: da = one + v * v; break;
    case O_TANH: da = one - v * v; break;
    case O_ATAN: da = one / (one + va * va); break;
    case O_FABS: da = va > zero ? one : (va < zero ? -one : zero); break;
    case O_FMIN: if (vb < va) { db = one; } else { da = one; } break;
    case O_FMAX: if (vb > va) { db = one; } else { da = one; } break;
    case O_LT: case O_LE: break;
    case O_POW: da = vb * std::pow(va, vb - one); db = std::log(va) * v; break;
    case O_ATAN2: { S r2 = va * va + vb * vb; da = vb / r2; db = -va / r2; } break;
    default: std::abort();
  }
  r.d.resize(K);
  for (int k = 0; k < K; ++k) {
    S t = zero;
    if (da != zero && a.d[k] != zero) t += da * a.d[k];
    if (use_b && db != zero && b.d[k] != zero) t += db * b.d[k];
    r.d[k] = t;
  }
  r.v = v;
}

// ------------------------------------------------------------ interpreter
struct Args {
  long long n;
  const double* const* in;
  const long long* ld_in;
  double* const* out;
  const long long* ld_out;
  // dual mode only
  int K;
  const double* tin;   // [K][tot_in][n]
  double* tout;        // [K][tot_out][n]
};

template <class S>
void run_range(const Prog& p, const Args& A, long long n0, long long n1) {
  std::vector<S> w(p.n_work);
  std::vector<S> cs(p.consts.size());
  for (size_t c = 0; c < cs.size(); ++c) cs[c] = s_const<S>(p.consts[c]);
  for (long long n = n0; n < n1; ++n) {
    for (const Instr& in : p.ins) {
      switch (in.op) {
        case O_INPUT: w[in.out] = (S)A.in[in.a][in.b * A.ld_in[in.a] + n]; break;
        case O_OUTPUT: A.out[in.out][in.b * A.ld_out[in.out] + n] = (double)w[in.a]; break;
        case O_CONST: w[in.out] = cs[in.a]; break;
        default: {
          S a = w[in.a];
          S b = binary(in.op) ? w[in.b] : S(0);
          if (in.f32) {
            // operands rounded to binary32, operation in binary32, result widened
            float r = apply<float>(in.op, (float)a, (float)b);
            w[in.out] = (S)r;
          } else {
            w[in.out] = apply<S>(in.op, a, b);
          }
        }
      }
    }
  }
}

template <class S>
void run_range_dual(const Prog& p, const Args& A, long long n0, long long n1) {
  const int K = A.K;
  std::vector<Dual<S>> w(p.n_work);
  Dual<S> zero;
  zero.v = S(0);
  zero.d.assign(K, S(0));
  for (long long n = n0; n < n1; ++n) {
    for (const Instr& in : p.ins) {
      switch (in.op) {
        case O_INPUT: {
          Dual<S>& r = w[in.out];
          r.v = (S)A.in[in.a][in.b * A.ld_in[in.a] + n];
          r.d.resize(K);
          long long e = p.off_in[in.a] + in.b;
          for (int k = 0; k < K; ++k) r.d[k] = (S)A.tin[((long long)k * p.tot_in + e) * A.n + n];
          break;
        }
        case O_OUTPUT: {
          const Dual<S>& s = w[in.a];
          A.out[in.out][in.b * A.ld_out[in.out] + n] = (double)s.v;
          long long e = p.off_out[in.out] + in.b;
          for (int k = 0; k < K; ++k) A.tout[((long long)k * p.tot_out + e) * A.n + n] = (double)s.d[k];
          break;
        }
        case O_CONST: {
          Dual<S>& r = w[in.out];
          r.v = (S)p.consts[in.a];
          r.d.assign(K, S(0));
          break;
        }
        default: {
          Dual<S> r;
          dual_apply<S>(in.op, w[in.a], binary(in.op) ? w[in.b] : zero, r, K);
          if (in.f32)  // value as the interpreter computes it
            r.v = (S)apply<float>(in.op, (float)w[in.a].v, binary(in.op) ? (float)w[in.b].v : 0.0f);
          w[in.out] = std::move(r);
        }
      }
    }
  }
}

template <class F>
void parallel(long long n, int threads, F f) {
  if (threads < 1) threads = 1;
  if (threads > n) threads = (int)(n > 0 ? n : 1);
  std::vector<std::thread> ts;
  long long chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    long long a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    ts.emplace_back([=] { f(a, b); });
  }
  for (auto& t : ts) t.join();
}

thread_local std::string g_err;

}  // namespace

extern "C" {

// Load and validate a program file.  Returns 0 and a handle, or -1 (see
// xo_last_error).
int xo_load(const char* path, void** handle) {
  Prog* p = new Prog();
  std::string err;
  if (!parse(path, *p, err) || !validate(*p, err)) {
    g_err = err;
    delete p;
    *handle = nullptr;
    return -1;
  }
  *handle = p;
  return 0;
}

void xo_free(void* h) { delete static_cast<Prog*>(h); }

const char* xo_last_error(void) { return g_err.c_str(); }

// Sizes: returns n_in, n_out; fills nnz arrays if non-null (caller sizes them).
int xo_info(void* h, long long* n_in, long long* n_out, long long* nnz_in, long long* nnz_out,
            long long* n_work, long long* n_instr) {
  const Prog* p = static_cast<Prog*>(h);
  *n_in = (long long)p->nnz_in.size();
  *n_out = (long long)p->nnz_out.size();
  if (nnz_in) for (size_t a = 0; a < p->nnz_in.size(); ++a) nnz_in[a] = p->nnz_in[a];
  if (nnz_out) for (size_t a = 0; a < p->nnz_out.size(); ++a) nnz_out[a] = p->nnz_out[a];
  if (n_work) *n_work = p->n_work;
  if (n_instr) *n_instr = (long long)p->ins.size();
  return 0;
}

// Evaluate for n instances.  scalar: 32 = float, 64 = double, 80 = long
// double.  Argument a, element e, instance i lives at ptr[a][e*ld[a] + i]
// (inputs are read as double and rounded once to the scalar type; outputs
// are rounded once to double).  Instances are split statically over
// `threads` std::threads.
int xo_eval(void* h, int scalar, long long n, const double* const* in, const long long* ld_in,
            double* const* out, const long long* ld_out, int threads) {
  const Prog& p = *static_cast<Prog*>(h);
  Args A{n, in, ld_in, out, ld_out, 0, nullptr, nullptr};
  if (scalar == 32) parallel(n, threads, [&](long long a, long long b) { run_range<float>(p, A, a, b); });
  else if (scalar == 64) parallel(n, threads, [&](long long a, long long b) { run_range<double>(p, A, a, b); });
  else if (scalar == 80) parallel(n, threads, [&](long long a, long long b) { run_range<long double>(p, A, a, b); });
  else { g_err = "scalar must be 32, 64 or 80"; return -1; }
  return 0;
}

// Forward-mode derivatives with dual numbers: K tangent directions, in
// scalar type 64 (double) or 32 (float: inputs and tangents rounded once to
// binary32, every operation in binary32).  tin[k][e][i] is the tangent of
// flattened input element e (args concatenated) for direction k and
// instance i; tout likewise for outputs.  Values are written to `out`
// exactly as xo_eval with the same scalar would.
int xo_jvp(void* h, int scalar, long long n, const double* const* in, const long long* ld_in,
           double* const* out, const long long* ld_out, int K, const double* tin, double* tout,
           int threads) {
  const Prog& p = *static_cast<Prog*>(h);
  if (K < 1) { g_err = "K must be >= 1"; return -1; }
  Args A{n, in, ld_in, out, ld_out, K, tin, tout};
  if (scalar == 64) parallel(n, threads, [&](long long a, long long b) { run_range_dual<double>(p, A, a, b); });
  else if (scalar == 32) parallel(n, threads, [&](long long a, long long b) { run_range_dual<float>(p, A, a, b); });
  else { g_err = "scalar must be 32 or 64"; return -1; }
  return 0;
}

}  // extern "C"
