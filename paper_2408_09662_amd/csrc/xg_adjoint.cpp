// Reverse-mode adjoint of an SSA program, built as another straight-line
// program (source transformation), so it is compiled and evaluated by the
// same planner and emitter as any forward program.
//
// The paper obtains derivatives symbolically in its front end before code
// generation (background section on algorithmic differentiation); here the
// library derives them itself from the loaded program.  For x_bar =
// J(x)^T y_bar the reverse sweep needs the forward values in reverse order.
// Keeping all of them (a tape) would hold every intermediate per instance;
// instead the forward sweep runs once, and the program is reversed range by
// range, recursively: a range is cut where few values are live, the states
// at its cuts are computed, and its parts are reversed last to first, each
// recomputed from the state at its start (checkpointing with recomputation,
// nested: only the states on the current path of the recursion are held).
#include <algorithm>
#include <climits>
#include <cstring>
#include <functional>
#include <unordered_map>

#include "xg_internal.h"

namespace xg {

namespace {

struct Builder {
  Graph G;
  std::unordered_map<uint64_t, int32_t> constmap;
  // unary nodes available in the current segment: (op, operand) -> node,
  // so a derivative such as cos(a) for sin(a) reuses a value the segment
  // already computes
  std::unordered_map<uint64_t, int32_t> unary;

  int32_t add(uint8_t op, int32_t a, int32_t b, int64_t aux = 0) {
    Node n;
    n.op = op; n.a = a; n.b = b; n.aux = aux;
    G.nodes.push_back(n);
    return (int32_t)G.nodes.size() - 1;
  }
  int32_t cst(double v) {
    uint64_t bits;
    std::memcpy(&bits, &v, 8);
    auto it = constmap.find(bits);
    if (it != constmap.end()) return it->second;
    G.consts.push_back(v);
    int32_t id = add(XG_OP_CONST, -1, -1, (int64_t)G.consts.size() - 1);
    constmap[bits] = id;
    return id;
  }
  int32_t bin(uint8_t op, int32_t a, int32_t b) { return add(op, a, b); }
  int32_t un(uint8_t op, int32_t a) { return add(op, a, -1); }
  static uint64_t ukey(uint8_t op, int32_t a) { return ((uint64_t)op << 32) | (uint32_t)a; }
  int32_t un_cse(uint8_t op, int32_t a) {
    auto it = unary.find(ukey(op, a));
    if (it != unary.end()) return it->second;
    int32_t v = add(op, a, -1);
    unary[ukey(op, a)] = v;
    return v;
  }
};

}  // namespace

Graph adjoint(const Graph& g, bool with_primal, int seg_ops, int64_t* recompute_ops, int fanout) {
  Builder B;
  B.G.dtype = g.dtype;
  B.G.consts = g.consts;  // constants of g keep their indices
  B.G.nnz_in = g.nnz_in;
  for (int32_t k : g.nnz_out) B.G.nnz_in.push_back(k);  // seeds
  const int32_t n_in = (int32_t)g.nnz_in.size();
  const int32_t n = (int32_t)g.nodes.size();
  if (fanout < 2) fanout = 2;

  // forward sweep: copy g
  std::vector<int32_t> fwd(n);
  for (int32_t i = 0; i < n; ++i) {
    Node nd = g.nodes[i];
    if (nd.a >= 0) nd.a = fwd[nd.a];
    if (nd.b >= 0) nd.b = fwd[nd.b];
    B.G.nodes.push_back(nd);
    fwd[i] = (int32_t)B.G.nodes.size() - 1;
    if (nd.op == XG_OP_CONST) {
      uint64_t bits;
      std::memcpy(&bits, &g.consts[nd.aux], 8);
      B.constmap.emplace(bits, fwd[i]);
    }
  }

  // The reverse sweep walks the program in a low-register-pressure order.
  // Ranges of that order are reversed recursively: a range of more than
  // seg_ops operations is cut into up to `fanout` parts where the fewest
  // values are live; the states at the cuts are computed (a forward pass
  // over all parts but the last, or taken from the forward sweep), then the
  // parts are reversed last to first, each from the state at its start.  A
  // range of at most seg_ops operations (a leaf) is recomputed from the
  // state at its start, then its adjoints are propagated.  Only the states
  // at the cuts on the current path of the recursion are held, never every
  // value crossing some cut: checkpoints at small live sets, recomputation
  // in between (one more forward pass of a range per level).
  const std::vector<int32_t> seq = low_pressure_order(g);
  const int32_t L = (int32_t)seq.size();
  std::vector<int32_t> ops_before(L + 1, 0);
  for (int32_t p = 0; p < L; ++p) ops_before[p + 1] = ops_before[p] + (is_arith(g.nodes[seq[p]].op) ? 1 : 0);
  // live_after[p]: values computed at positions <= p read after p (inputs
  // and constants are reloaded, never held)
  std::vector<int32_t> live_after(L, 0);
  {
    std::vector<int32_t> pos(n, -1), last(n, -1);
    for (int32_t p = 0; p < L; ++p) pos[seq[p]] = p;
    for (int32_t p = 0; p < L; ++p) {
      const Node& nd = g.nodes[seq[p]];
      if (nd.a >= 0) last[nd.a] = std::max(last[nd.a], p);
      if (nd.b >= 0) last[nd.b] = std::max(last[nd.b], p);
    }
    std::vector<int32_t> ends(L + 1, 0);
    int32_t live = 0;
    for (int32_t p = 0; p < L; ++p) {
      const int32_t v = seq[p];
      const uint8_t op = g.nodes[v].op;
      if (op != XG_OP_INPUT && last[v] > p) { live++; ends[last[v]]++; }
      live -= ends[p];
      live_after[p] = live;
    }
  }

  // current version (node id in B.G) of every value of g
  std::vector<int32_t> cur = fwd;
  // adjoint accumulators (node ids in B.G), -1 = structurally zero
  std::vector<int32_t> adj(n, -1);
  auto acc = [&](int32_t k, int32_t term, bool negate) {
    if (g.nodes[k].op == XG_OP_CONST) return;
    if (adj[k] < 0) adj[k] = negate ? B.un(XG_OP_NEG, term) : term;
    else adj[k] = B.bin(negate ? XG_OP_SUB : XG_OP_ADD, adj[k], term);
  };
  // seeds
  for (int32_t a = 0; a < (int32_t)g.out.size(); ++a)
    for (int32_t e = 0; e < (int32_t)g.out[a].size(); ++e) {
      int32_t s = B.add(XG_OP_INPUT, -1, -1, ((int64_t)(n_in + a) << 32) | (uint32_t)e);
      acc(g.out[a][e], s, false);
    }

  int64_t nrec = 0;
  // recompute positions [p0, p1) from the current versions of their operands
  auto recompute = [&](int32_t p0, int32_t p1) {
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t i = seq[p];
      const Node& nd = g.nodes[i];
      if (nd.op == XG_OP_INPUT) { cur[i] = fwd[i]; continue; }  // reloaded, not recomputed
      cur[i] = B.add(nd.op, nd.a >= 0 ? cur[nd.a] : -1, nd.b >= 0 ? cur[nd.b] : -1, nd.aux);
      B.G.nodes[cur[i]].f32 = nd.f32;  // recomputed exactly as in the forward sweep
      ++nrec;
    }
  };
  // propagate adjoints through the operation at position p (values: cur)
  auto reverse_op = [&](int32_t p) {
    const int32_t i = seq[p];
    const int32_t w = adj[i];
    if (w < 0) return;
    const Node& nd = g.nodes[i];
    if (nd.op == XG_OP_INPUT || nd.op == XG_OP_CONST) return;
    const int32_t A = nd.a >= 0 ? cur[nd.a] : -1;
    const int32_t Bv = nd.b >= 0 ? cur[nd.b] : -1;
    const int32_t V = cur[i];
    const bool ca = nd.a >= 0 && g.nodes[nd.a].op == XG_OP_CONST;
    const bool cb = nd.b >= 0 && g.nodes[nd.b].op == XG_OP_CONST;
    switch (nd.op) {
      case XG_OP_ADD: acc(nd.a, w, false); acc(nd.b, w, false); break;
      case XG_OP_SUB: acc(nd.a, w, false); acc(nd.b, w, true); break;
      case XG_OP_MUL:
        if (!ca) acc(nd.a, B.bin(XG_OP_MUL, w, Bv), false);
        if (!cb) acc(nd.b, B.bin(XG_OP_MUL, w, A), false);
        break;
      case XG_OP_DIV: {
        int32_t t = B.bin(XG_OP_DIV, w, Bv);
        if (!ca) acc(nd.a, t, false);
        if (!cb) acc(nd.b, B.bin(XG_OP_MUL, t, V), true);
        break;
      }
      case XG_OP_NEG: acc(nd.a, w, true); break;
      case XG_OP_ASSIGN: acc(nd.a, w, false); break;
      case XG_OP_SQ: {
        int32_t t = B.bin(XG_OP_MUL, w, A);
        acc(nd.a, B.bin(XG_OP_ADD, t, t), false);
        break;
      }
      case XG_OP_SQRT:
        acc(nd.a, B.bin(XG_OP_DIV, B.bin(XG_OP_MUL, w, B.cst(0.5)), V), false);
        break;
      case XG_OP_EXP: acc(nd.a, B.bin(XG_OP_MUL, w, V), false); break;
      case XG_OP_LOG: acc(nd.a, B.bin(XG_OP_DIV, w, A), false); break;
      case XG_OP_SIN: acc(nd.a, B.bin(XG_OP_MUL, w, B.un_cse(XG_OP_COS, A)), false); break;
      case XG_OP_COS: acc(nd.a, B.bin(XG_OP_MUL, w, B.un_cse(XG_OP_SIN, A)), true); break;
      case XG_OP_TAN:
        acc(nd.a, B.bin(XG_OP_MUL, w, B.bin(XG_OP_ADD, B.cst(1.0), B.bin(XG_OP_MUL, V, V))), false);
        break;
      case XG_OP_TANH:
        acc(nd.a, B.bin(XG_OP_MUL, w, B.bin(XG_OP_SUB, B.cst(1.0), B.bin(XG_OP_MUL, V, V))), false);
        break;
      case XG_OP_ATAN:
        acc(nd.a, B.bin(XG_OP_DIV, w, B.bin(XG_OP_ADD, B.cst(1.0), B.bin(XG_OP_MUL, A, A))), false);
        break;
      case XG_OP_FABS: {
        // sign(a) with sign(0) = 0
        int32_t z = B.cst(0.0);
        int32_t sg = B.bin(XG_OP_SUB, B.bin(XG_OP_LT, z, A), B.bin(XG_OP_LT, A, z));
        acc(nd.a, B.bin(XG_OP_MUL, w, sg), false);
        break;
      }
      case XG_OP_FMIN: case XG_OP_FMAX: {
        // the second operand is chosen only when strictly better; a tie
        // goes to the first
        int32_t pick_b = nd.op == XG_OP_FMIN ? B.bin(XG_OP_LT, Bv, A) : B.bin(XG_OP_LT, A, Bv);
        if (!ca) acc(nd.a, B.bin(XG_OP_MUL, w, B.bin(XG_OP_SUB, B.cst(1.0), pick_b)), false);
        if (!cb) acc(nd.b, B.bin(XG_OP_MUL, w, pick_b), false);
        break;
      }
      case XG_OP_LT: case XG_OP_LE: break;
      case XG_OP_POW: {
        if (!ca) {
          int32_t p1 = B.bin(XG_OP_POW, A, B.bin(XG_OP_SUB, Bv, B.cst(1.0)));
          acc(nd.a, B.bin(XG_OP_MUL, w, B.bin(XG_OP_MUL, Bv, p1)), false);
        }
        if (!cb) acc(nd.b, B.bin(XG_OP_MUL, w, B.bin(XG_OP_MUL, B.un(XG_OP_LOG, A), V)), false);
        break;
      }
      case XG_OP_ATAN2: {
        int32_t r2 = B.bin(XG_OP_ADD, B.bin(XG_OP_MUL, A, A), B.bin(XG_OP_MUL, Bv, Bv));
        int32_t t = B.bin(XG_OP_DIV, w, r2);
        if (!ca) acc(nd.a, B.bin(XG_OP_MUL, t, Bv), false);
        if (!cb) acc(nd.b, B.bin(XG_OP_MUL, t, A), true);
        break;
      }
      default: break;
    }
  };
  auto leaf = [&](int32_t p0, int32_t p1, bool computed) {
    if (!computed) recompute(p0, p1);
    // derivative helpers such as cos(a) for sin(a) reuse a unary value the
    // leaf computes anyway
    B.unary.clear();
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t i = seq[p];
      const Node& nd = g.nodes[i];
      if (nd.a >= 0 && nd.b < 0 && is_arith(nd.op)) B.unary[Builder::ukey(nd.op, cur[nd.a])] = cur[i];
    }
    for (int32_t p = p1 - 1; p >= p0; --p) reverse_op(p);
  };
  const int32_t leaf_ops = seg_ops > 0 ? seg_ops : INT32_MAX;
  // reverse positions [p0, p1); `computed`: the current versions of its
  // values already exist (the forward sweep, for the program's last parts)
  std::function<void(int32_t, int32_t, bool)> rev = [&](int32_t p0, int32_t p1, bool computed) {
    const int32_t ops = ops_before[p1] - ops_before[p0];
    if (ops <= leaf_ops || p1 - p0 < 2) { leaf(p0, p1, computed); return; }
    const int32_t m = (int32_t)std::min<int64_t>(fanout, (ops + (int64_t)leaf_ops - 1) / leaf_ops);
    // cut k near k/m of the operations, at the fewest live values within
    // a quarter part either side
    std::vector<int32_t> cut = {p0};
    const int64_t part = ops / m, win = std::max<int64_t>(1, part / 4);
    for (int32_t k = 1; k < m; ++k) {
      const int64_t t = ops_before[p0] + part * k;
      int32_t best = -1, bl = INT32_MAX;
      for (int32_t q = cut.back() + 1; q < p1; ++q) {
        if (ops_before[q] < t - win) continue;
        if (ops_before[q] > t + win) break;
        if (live_after[q - 1] < bl) { bl = live_after[q - 1]; best = q; }
      }
      if (best > cut.back()) cut.push_back(best);
    }
    cut.push_back(p1);
    const int32_t parts = (int32_t)cut.size() - 1;
    if (parts < 2) { leaf(p0, p1, computed); return; }
    if (!computed) recompute(cut[0], cut[parts - 1]);  // the states at the cuts
    rev(cut[parts - 1], cut[parts], computed);
    for (int32_t j = parts - 2; j >= 0; --j) rev(cut[j], cut[j + 1], false);
  };
  rev(0, L, true);

  // outputs: gradients per input element, then (optionally) primal outputs
  std::vector<std::vector<int32_t>> in_node(n_in);
  for (int32_t a = 0; a < n_in; ++a) in_node[a].assign(g.nnz_in[a], -1);
  for (int32_t i = 0; i < n; ++i)
    if (g.nodes[i].op == XG_OP_INPUT) {
      int32_t a = (int32_t)(g.nodes[i].aux >> 32), e = (int32_t)(g.nodes[i].aux & 0xffffffff);
      in_node[a][e] = i;
    }
  for (int32_t a = 0; a < n_in; ++a) {
    B.G.nnz_out.push_back(g.nnz_in[a]);
    std::vector<int32_t> o(g.nnz_in[a]);
    for (int32_t e = 0; e < g.nnz_in[a]; ++e) {
      int32_t k = in_node[a][e];
      o[e] = (k >= 0 && adj[k] >= 0) ? adj[k] : B.cst(0.0);
    }
    B.G.out.push_back(o);
  }
  if (with_primal) {
    for (int32_t a = 0; a < (int32_t)g.out.size(); ++a) {
      B.G.nnz_out.push_back(g.nnz_out[a]);
      std::vector<int32_t> o(g.out[a].size());
      for (size_t e = 0; e < o.size(); ++e) o[e] = fwd[g.out[a][e]];
      B.G.out.push_back(o);
    }
  }
  if (recompute_ops) *recompute_ops = nrec;
  dce(B.G);
  return B.G;
}

}  // namespace xg
