// Test driver: the library's reverse-mode transformation (xg::adjoint) of a
// program, evaluated on the CPU by a plain sequential walk of its SSA nodes,
// so the transformation can be checked against the oracle's dual numbers
// without a GPU.
//
//   adjoint_eval <desc.txt> <seg_ops> <fanout> <inputs.bin> <outputs.bin>
//
// desc.txt: "dtype n_work n_in nnz.. n_out nnz.. n_const c.. n_instr
// (op out a b prec)..." (constants as C99 hex floats).  inputs.bin: N, then
// for every instance the adjoint program's inputs (the program's inputs,
// then one seed per output element), doubles.  outputs.bin: for every
// instance the adjoint program's outputs (gradients, then primal outputs),
// doubles; followed by the number of recomputed operations.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include "xg_internal.h"

namespace {

template <class S>
S apply(int op, S a, S b) {
  switch (op) {
    case XG_OP_ADD: return a + b;
    case XG_OP_SUB: return a - b;
    case XG_OP_MUL: return a * b;
    case XG_OP_DIV: return a / b;
    case XG_OP_NEG: return -a;
    case XG_OP_SQ: return a * a;
    case XG_OP_SQRT: return std::sqrt(a);
    case XG_OP_EXP: return std::exp(a);
    case XG_OP_LOG: return std::log(a);
    case XG_OP_SIN: return std::sin(a);
    case XG_OP_COS: return std::cos(a);
    case XG_OP_TAN: return std::tan(a);
    case XG_OP_TANH: return std::tanh(a);
    case XG_OP_ATAN: return std::atan(a);
    case XG_OP_FABS: return std::fabs(a);
    case XG_OP_FMIN: return std::fmin(a, b);
    case XG_OP_FMAX: return std::fmax(a, b);
    case XG_OP_LT: return a < b ? S(1) : S(0);
    case XG_OP_LE: return a <= b ? S(1) : S(0);
    case XG_OP_POW: return std::pow(a, b);
    case XG_OP_ATAN2: return std::atan2(a, b);
    case XG_OP_ASSIGN: return a;
  }
  std::abort();
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 6) return 2;
  std::ifstream f(argv[1]);
  int dtype, n_work, n_in, n_out, n_const;
  long long n_instr;
  f >> dtype >> n_work >> n_in;
  std::vector<int32_t> nnz_in(n_in);
  for (auto& v : nnz_in) f >> v;
  f >> n_out;
  std::vector<int32_t> nnz_out(n_out);
  for (auto& v : nnz_out) f >> v;
  f >> n_const;
  std::vector<double> consts(n_const);
  for (auto& c : consts) { std::string s; f >> s; c = std::strtod(s.c_str(), nullptr); }
  f >> n_instr;
  std::vector<xg_instr> ins(n_instr);
  std::vector<int8_t> prec(n_instr);
  for (auto& in : ins) { int p; f >> in.op >> in.out >> in.a >> in.b >> p; prec[&in - ins.data()] = (int8_t)p; }
  if (!f) return 2;
  xg_program_desc d{n_in, nnz_in.data(), n_out, nnz_out.data(), n_work, n_instr, ins.data(),
                    n_const, consts.data(), dtype, prec.data()};
  xg::Graph g;
  std::string err;
  if (!xg::build_graph(d, g, err)) { std::fprintf(stderr, "%s\n", err.c_str()); return 3; }
  int64_t nrec = 0;
  xg::Graph G = xg::adjoint(g, true, std::atoi(argv[2]), &nrec, std::atoi(argv[3]));
  std::ifstream fi(argv[4], std::ios::binary);
  long long N = 0;
  fi.read((char*)&N, 8);
  std::vector<long long> off(G.nnz_in.size() + 1, 0);
  for (size_t a = 0; a < G.nnz_in.size(); ++a) off[a + 1] = off[a] + G.nnz_in[a];
  std::vector<double> x(off.back()), w(G.nodes.size());
  std::ofstream fo(argv[5], std::ios::binary);
  for (long long i = 0; i < N; ++i) {
    fi.read((char*)x.data(), (std::streamsize)(8 * x.size()));
    if (!fi) return 4;
    for (size_t k = 0; k < G.nodes.size(); ++k) {
      const xg::Node& nd = G.nodes[k];
      if (nd.op == XG_OP_INPUT) w[k] = x[off[nd.aux >> 32] + (nd.aux & 0xffffffff)];
      else if (nd.op == XG_OP_CONST) w[k] = G.consts[nd.aux];
      else if (nd.f32 || G.dtype == XG_F32)
        w[k] = (double)apply<float>(nd.op, (float)w[nd.a], nd.b >= 0 ? (float)w[nd.b] : 0.0f);
      else w[k] = apply<double>(nd.op, w[nd.a], nd.b >= 0 ? w[nd.b] : 0.0);
    }
    for (auto& arg : G.out)
      for (int32_t v : arg) fo.write((const char*)&w[v], 8);
  }
  double r = (double)nrec;
  fo.write((const char*)&r, 8);
  return 0;
}
