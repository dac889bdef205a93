// Program validation and conversion to SSA.
//
// The input is the paper's work-vector form (section "Code Generation"):
// instructions over reusable slots, evaluated in order.  Each slot write
// becomes a new SSA value, so slot reuse (including in-place updates such
// as the listing's work[1] = work[1] + work[0]) disappears: an instruction
// reads the values its operand slots hold before it, then its output slot
// holds the new value.
#include <algorithm>
#include <cstring>
#include <unordered_map>

#include "xg_internal.h"

namespace xg {

static const char* kNames[XG_OP_COUNT] = {
    "INPUT", "OUTPUT", "CONST", "ASSIGN", "ADD", "SUB", "MUL", "DIV", "NEG",
    "SQ", "SQRT", "EXP", "LOG", "SIN", "COS", "TAN", "TANH", "ATAN",
    "FABS", "FMIN", "FMAX", "LT", "LE", "POW", "ATAN2"};

const char* op_name(int op) { return (op >= 0 && op < XG_OP_COUNT) ? kNames[op] : "?"; }

bool is_binary(int op) {
  switch (op) {
    case XG_OP_ADD: case XG_OP_SUB: case XG_OP_MUL: case XG_OP_DIV: case XG_OP_FMIN:
    case XG_OP_FMAX: case XG_OP_LT: case XG_OP_LE: case XG_OP_POW: case XG_OP_ATAN2:
      return true;
  }
  return false;
}

bool is_arith(int op) {
  return op != XG_OP_INPUT && op != XG_OP_OUTPUT && op != XG_OP_CONST && op != XG_OP_ASSIGN;
}

namespace {
struct Key {
  uint8_t op, f32;
  int32_t a, b;
  int64_t aux;
  bool operator==(const Key& o) const {
    return op == o.op && f32 == o.f32 && a == o.a && b == o.b && aux == o.aux;
  }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h ^= v; h *= 1099511628211ull; };
    mix(k.op); mix(k.f32); mix((uint32_t)k.a); mix((uint32_t)k.b); mix((uint64_t)k.aux);
    return (size_t)h;
  }
};
}  // namespace

bool build_graph(const xg_program_desc& d, Graph& g, std::string& err) {
  if (d.dtype != XG_F32 && d.dtype != XG_F64) { err = "dtype must be XG_F32 or XG_F64"; return false; }
  if (d.n_in < 0 || d.n_out < 0 || d.n_work < 0 || d.n_instr < 0 || d.n_const < 0) {
    err = "negative size in program description"; return false;
  }
  if ((d.n_in && !d.nnz_in) || (d.n_out && !d.nnz_out) || (d.n_instr && !d.instr) ||
      (d.n_const && !d.consts)) {
    err = "null array in program description"; return false;
  }
  g = Graph();
  g.dtype = d.dtype;
  g.nnz_in.assign(d.nnz_in, d.nnz_in + d.n_in);
  g.nnz_out.assign(d.nnz_out, d.nnz_out + d.n_out);
  for (int32_t v : g.nnz_in) if (v < 0) { err = "negative nnz_in"; return false; }
  for (int32_t v : g.nnz_out) if (v < 0) { err = "negative nnz_out"; return false; }
  g.consts.assign(d.consts, d.consts + d.n_const);
  g.out.resize(d.n_out);
  for (int32_t a = 0; a < d.n_out; ++a) g.out[a].assign(g.nnz_out[a], -1);
  std::vector<int32_t> slot(d.n_work, -1);
  std::unordered_map<Key, int32_t, KeyHash> memo;
  auto node = [&](uint8_t op, int32_t a, int32_t b, int64_t aux, uint8_t f32) -> int32_t {
    if ((op == XG_OP_ADD || op == XG_OP_MUL) && a > b) std::swap(a, b);
    Key k{op, f32, a, b, aux};
    auto it = memo.find(k);
    if (it != memo.end()) return it->second;
    int32_t id = (int32_t)g.nodes.size();
    Node n;
    n.op = op; n.f32 = f32; n.a = a; n.b = b; n.aux = aux;
    g.nodes.push_back(n);
    memo.emplace(k, id);
    return id;
  };
  for (int64_t i = 0; i < d.n_instr; ++i) {
    const xg_instr& in = d.instr[i];
    std::string at = " at instruction " + std::to_string(i);
    if (in.op < 0 || in.op >= XG_OP_COUNT) { err = "unknown op " + std::to_string(in.op) + at; return false; }
    auto rd = [&](int32_t s, int32_t& v) {
      if (s < 0 || s >= d.n_work) { err = "slot out of range" + at; return false; }
      if (slot[s] < 0) { err = "read before write" + at; return false; }
      v = slot[s];
      return true;
    };
    int32_t va = -1, vb = -1, res = -1;
    switch (in.op) {
      case XG_OP_INPUT:
        if (in.a < 0 || in.a >= d.n_in || in.b < 0 || in.b >= g.nnz_in[in.a]) {
          err = "input index out of range" + at; return false;
        }
        res = node(XG_OP_INPUT, -1, -1, ((int64_t)in.a << 32) | (uint32_t)in.b, 0);
        break;
      case XG_OP_CONST:
        if (in.a < 0 || in.a >= d.n_const) { err = "const index out of range" + at; return false; }
        res = node(XG_OP_CONST, -1, -1, in.a, 0);
        break;
      case XG_OP_OUTPUT:
        if (in.out < 0 || in.out >= d.n_out || in.b < 0 || in.b >= g.nnz_out[in.out]) {
          err = "output index out of range" + at; return false;
        }
        if (!rd(in.a, va)) return false;
        g.out[in.out][in.b] = va;  // last write wins
        continue;
      case XG_OP_ASSIGN:
        if (!rd(in.a, va)) return false;
        res = va;
        break;
      default: {
        if (!rd(in.a, va)) return false;
        if (is_binary(in.op) && !rd(in.b, vb)) return false;
        uint8_t f32 = 0;
        if (d.prec && d.prec[i] != 0) {
          if (d.prec[i] == 32 && d.dtype == XG_F64) f32 = 1;
          else if (!(d.prec[i] == 64 && d.dtype == XG_F64) && !(d.prec[i] == 32 && d.dtype == XG_F32)) {
            err = "precision tag must be 0, 32 (in an f64 program) or the program's own" + at;
            return false;
          }
        }
        res = node((uint8_t)in.op, va, is_binary(in.op) ? vb : -1, 0, f32);
      }
    }
    if (in.out < 0 || in.out >= d.n_work) { err = "slot out of range" + at; return false; }
    slot[in.out] = res;
  }
  for (size_t a = 0; a < g.out.size(); ++a)
    for (size_t e = 0; e < g.out[a].size(); ++e)
      if (g.out[a][e] < 0) {
        err = "output " + std::to_string(a) + "[" + std::to_string(e) + "] never written";
        return false;
      }
  dce(g);
  return true;
}

void dce(Graph& g) {
  const int32_t n = (int32_t)g.nodes.size();
  std::vector<char> live(n, 0);
  for (auto& arg : g.out) for (int32_t v : arg) live[v] = 1;
  for (int32_t i = n - 1; i >= 0; --i) {
    if (!live[i]) continue;
    const Node& nd = g.nodes[i];
    if (nd.a >= 0) live[nd.a] = 1;
    if (nd.b >= 0) live[nd.b] = 1;
  }
  std::vector<int32_t> remap(n, -1);
  std::vector<Node> nodes;
  nodes.reserve(n);
  for (int32_t i = 0; i < n; ++i) {
    if (!live[i]) continue;
    Node nd = g.nodes[i];
    if (nd.a >= 0) nd.a = remap[nd.a];
    if (nd.b >= 0) nd.b = remap[nd.b];
    remap[i] = (int32_t)nodes.size();
    nodes.push_back(nd);
  }
  g.nodes.swap(nodes);
  for (auto& arg : g.out) for (int32_t& v : arg) v = remap[v];
}

void cse(Graph& g) {
  std::unordered_map<Key, int32_t, KeyHash> memo;
  const int32_t n = (int32_t)g.nodes.size();
  std::vector<int32_t> rep(n);
  std::vector<Node> nodes;
  nodes.reserve(n);
  for (int32_t i = 0; i < n; ++i) {
    Node nd = g.nodes[i];
    if (nd.a >= 0) nd.a = rep[nd.a];
    if (nd.b >= 0) nd.b = rep[nd.b];
    if ((nd.op == XG_OP_ADD || nd.op == XG_OP_MUL) && nd.a > nd.b) std::swap(nd.a, nd.b);
    Key k{nd.op, nd.f32, nd.a, nd.b, nd.aux};
    auto it = memo.find(k);
    if (it != memo.end()) { rep[i] = it->second; continue; }
    rep[i] = (int32_t)nodes.size();
    memo.emplace(k, rep[i]);
    nodes.push_back(nd);
  }
  g.nodes.swap(nodes);
  for (auto& arg : g.out) for (int32_t& v : arg) v = rep[v];
}

int64_t share_reciprocals(Graph& g) {
  const int32_t n = (int32_t)g.nodes.size();
  // divisions per (divisor, precision tag)
  std::unordered_map<int64_t, int32_t> uses;
  auto key = [](int32_t b, uint8_t f32) { return ((int64_t)b << 1) | f32; };
  for (const Node& nd : g.nodes)
    if (nd.op == XG_OP_DIV) uses[key(nd.b, nd.f32)]++;
  int64_t shared = 0;
  for (auto& kv : uses) if (kv.second > 1) shared += kv.second;
  if (shared == 0) return 0;
  // the constant 1.0
  int32_t one_c = -1;
  for (size_t i = 0; i < g.consts.size(); ++i)
    if (g.consts[i] == 1.0) { one_c = (int32_t)i; break; }
  if (one_c < 0) { one_c = (int32_t)g.consts.size(); g.consts.push_back(1.0); }
  std::vector<Node> nodes;
  nodes.reserve(n + n / 8 + 2);
  std::vector<int32_t> remap(n, -1);
  int32_t one = -1;
  std::unordered_map<int64_t, int32_t> recip;  // (new divisor id, tag) -> reciprocal node
  int64_t replaced = 0;
  for (int32_t i = 0; i < n; ++i) {
    Node nd = g.nodes[i];
    if (nd.a >= 0) nd.a = remap[nd.a];
    if (nd.b >= 0) nd.b = remap[nd.b];
    if (g.nodes[i].op == XG_OP_DIV && uses[key(g.nodes[i].b, nd.f32)] > 1) {
      if (one < 0) {
        Node c;
        c.op = XG_OP_CONST; c.a = -1; c.b = -1; c.aux = one_c; c.f32 = 0;
        one = (int32_t)nodes.size();
        nodes.push_back(c);
      }
      const int64_t k = key(nd.b, nd.f32);
      auto it = recip.find(k);
      int32_t r;
      if (it == recip.end()) {
        Node q;
        q.op = XG_OP_DIV; q.a = one; q.b = nd.b; q.aux = 0; q.f32 = nd.f32;
        r = (int32_t)nodes.size();
        nodes.push_back(q);
        recip.emplace(k, r);
      } else {
        r = it->second;
      }
      ++replaced;
      const Node& num = g.nodes[g.nodes[i].a];
      if (num.op == XG_OP_CONST && g.consts[num.aux] == 1.0) {  // 1 / b is the reciprocal itself
        remap[i] = r;
        continue;
      }
      nd.op = XG_OP_MUL;
      nd.b = r;
      if (nd.a > nd.b) std::swap(nd.a, nd.b);
    }
    remap[i] = (int32_t)nodes.size();
    nodes.push_back(nd);
  }
  g.nodes.swap(nodes);
  for (auto& arg : g.out) for (int32_t& v : arg) v = remap[v];
  return replaced;
}

}  // namespace xg
