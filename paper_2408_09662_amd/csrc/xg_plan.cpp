// Scheduling, liveness and chunking of an SSA program.
//
// The paper's kernel keeps the whole work vector in global memory with one
// slot per intermediate (AoS, stride n_w) and lets the instruction order
// of the symbolic front end stand.  Here the order is chosen to keep the
// live set small, since live values are what must sit in registers:
// candidates are the front end's order and a greedy pressure-aware list
// schedule (prefer the ready operation that ends the most live ranges),
// and the one with the smaller maximum live set wins.  Very large programs
// are cut into chunks (one kernel each) at positions where few values are
// live; values that cross a cut go to a structure-of-arrays workspace.
#include <algorithm>
#include <queue>
#include <stdexcept>

#include "xg_internal.h"

namespace xg {

namespace {

// Distinct non-constant operands of node i.
inline int operands(const Graph& g, int32_t i, int32_t ops[2]) {
  const Node& nd = g.nodes[i];
  int k = 0;
  if (nd.a >= 0 && g.nodes[nd.a].op != XG_OP_CONST) ops[k++] = nd.a;
  if (nd.b >= 0 && nd.b != nd.a && g.nodes[nd.b].op != XG_OP_CONST) ops[k++] = nd.b;
  return k;
}

std::vector<int32_t> original_order(const Graph& g) {
  std::vector<int32_t> o;
  for (int32_t i = 0; i < (int32_t)g.nodes.size(); ++i)
    if (g.nodes[i].op != XG_OP_CONST) o.push_back(i);
  return o;
}

// Greedy top-down list schedule minimising register pressure.
std::vector<int32_t> greedy_order(const Graph& g) {
  const int32_t n = (int32_t)g.nodes.size();
  std::vector<std::vector<int32_t>> cons(n);
  std::vector<int32_t> pending(n, 0), remaining(n, 0);
  for (int32_t i = 0; i < n; ++i) {
    if (g.nodes[i].op == XG_OP_CONST) continue;
    int32_t ops[2];
    int k = operands(g, i, ops);
    pending[i] = k;
    for (int j = 0; j < k; ++j) { cons[ops[j]].push_back(i); remaining[ops[j]]++; }
  }
  std::vector<char> done(n, 0);
  auto score = [&](int32_t i) {
    int32_t ops[2];
    int k = operands(g, i, ops);
    int s = 0;
    for (int j = 0; j < k; ++j) if (remaining[ops[j]] == 1) ++s;
    if (!cons[i].empty()) s -= 1;
    return s + 1;  // 0..3
  };
  typedef std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> MinQ;
  MinQ q[4];
  std::vector<int8_t> cur(n, -1);
  auto push = [&](int32_t i) {
    int s = score(i);
    cur[i] = (int8_t)s;
    q[s].push(i);
  };
  for (int32_t i = 0; i < n; ++i)
    if (g.nodes[i].op != XG_OP_CONST && pending[i] == 0) push(i);
  std::vector<int32_t> order;
  order.reserve(n);
  while (true) {
    int32_t pick = -1;
    for (int s = 3; s >= 0 && pick < 0; --s) {
      while (!q[s].empty()) {
        int32_t i = q[s].top();
        q[s].pop();
        if (done[i] || cur[i] != s) continue;  // stale entry
        pick = i;
        break;
      }
    }
    if (pick < 0) break;
    done[pick] = 1;
    order.push_back(pick);
    int32_t ops[2];
    int k = operands(g, pick, ops);
    for (int j = 0; j < k; ++j) {
      int32_t v = ops[j];
      if (--remaining[v] == 1) {
        for (int32_t c : cons[v])
          if (!done[c] && pending[c] == 0) { push(c); break; }
      }
    }
    for (int32_t c : cons[pick])
      if (--pending[c] == 0) push(c);
  }
  return order;
}

}  // namespace

std::vector<int32_t> low_pressure_order(const Graph& g) {
  std::vector<int32_t> o1 = original_order(g);
  std::vector<int32_t> o2 = greedy_order(g);
  if (o2.size() == o1.size() && max_live_of(g, o2) < max_live_of(g, o1)) return o2;
  return o1;
}

int64_t max_live_of(const Graph& g, const std::vector<int32_t>& order) {
  const int32_t n = (int32_t)g.nodes.size();
  std::vector<int32_t> last(n, -1);
  for (int32_t p = 0; p < (int32_t)order.size(); ++p) {
    int32_t ops[2];
    int k = operands(g, order[p], ops);
    for (int j = 0; j < k; ++j) last[ops[j]] = p;
  }
  std::vector<int32_t> ends(order.size() + 1, 0);
  int64_t live = 0, best = 0;
  for (int32_t p = 0; p < (int32_t)order.size(); ++p) {
    int32_t v = order[p];
    if (last[v] > p) { live++; ends[last[v]]++; }
    best = std::max(best, live);
    live -= ends[p];
  }
  return best;
}

int op_cost(int op) {
  switch (op) {
    case XG_OP_DIV: return 10;
    case XG_OP_SQRT: return 8;
    case XG_OP_SIN: case XG_OP_COS: case XG_OP_TAN: case XG_OP_EXP: case XG_OP_LOG:
    case XG_OP_TANH: case XG_OP_ATAN: case XG_OP_POW: case XG_OP_ATAN2: return 40;
    case XG_OP_INPUT: case XG_OP_OUTPUT: case XG_OP_CONST: case XG_OP_ASSIGN: return 0;
  }
  return 1;
}

// Cooperative-tile plan: operations are grouped by dependency level (the
// longest chain of operations leading to them); a level with enough work
// is split over the W waves (contiguous runs of node ids, balanced by
// cost), consecutive levels with little work run on wave 0 alone with no
// barrier between them.
static Plan make_wide_plan(const Graph& g, const PlanOptions& po) {
  Plan pl;
  const int32_t n = (int32_t)g.nodes.size();
  const int W = po.waves;
  pl.waves = W;
  std::vector<int32_t> lvl(n, 0);
  int32_t depth = 0;
  for (int32_t v = 0; v < n; ++v) {
    const Node& nd = g.nodes[v];
    if (nd.op == XG_OP_CONST || nd.op == XG_OP_INPUT) continue;
    int32_t ops[2];
    int k = operands(g, v, ops);
    int32_t l = 0;
    for (int j = 0; j < k; ++j) l = std::max(l, lvl[ops[j]]);
    lvl[v] = l + 1;
    depth = std::max(depth, l + 1);
    pl.n_ops++;
  }
  pl.depth = depth;
  std::vector<std::vector<int32_t>> at(depth + 1);
  std::vector<int64_t> cost(depth + 1, 0);
  for (int32_t v = 0; v < n; ++v) {
    if (g.nodes[v].op == XG_OP_CONST) continue;
    at[lvl[v]].push_back(v);
    if (g.nodes[v].op != XG_OP_INPUT) cost[lvl[v]] += op_cost(g.nodes[v].op);
  }
  const int64_t narrow = 16 * (int64_t)W;  // below this a level runs on one wave
  std::vector<int32_t> chunk_of_node(n, -1);
  auto open_chunk = [&](int32_t phase, int32_t wave) {
    pl.chunks.push_back({(int32_t)pl.order.size(), (int32_t)pl.order.size()});
    pl.chunk_phase.push_back(phase);
    pl.chunk_wave.push_back(wave);
  };
  auto put = [&](int32_t v) {
    chunk_of_node[v] = (int32_t)pl.chunks.size() - 1;
    pl.order.push_back(v);
    pl.chunks.back().end = (int32_t)pl.order.size();
  };
  int32_t phase = 0;
  bool prev_narrow = false;
  open_chunk(0, 0);
  for (int32_t v : at[0]) put(v);  // inputs: loaded where used
  prev_narrow = true;
  for (int32_t l = 1; l <= depth; ++l) {
    if (cost[l] < narrow) {
      if (!prev_narrow) { ++phase; open_chunk(phase, 0); }
      for (int32_t v : at[l]) put(v);
      prev_narrow = true;
      continue;
    }
    ++phase;
    const int64_t target = (cost[l] + W - 1) / W;
    int64_t acc = 0;
    int w = 0;
    open_chunk(phase, 0);
    for (int32_t v : at[l]) {
      const int64_t c = op_cost(g.nodes[v].op);
      if (acc >= target * (w + 1) && w + 1 < W) { ++w; open_chunk(phase, w); }
      put(v);
      acc += c;
    }
    prev_narrow = false;
  }
  pl.n_phases = phase + 1;
  // live set of the order (informational)
  pl.max_live = max_live_of(g, pl.order);
  // values read outside their chunk -> workspace slots; a slot is reused
  // only by a value defined in a later phase than the last read of its
  // previous occupant (chunks of one phase run concurrently)
  pl.ws_slot.assign(n, -1);
  std::vector<int32_t> last_phase(n, -1);
  std::vector<char> crosses(n, 0);
  for (size_t c = 0; c < pl.chunks.size(); ++c)
    for (int32_t p = pl.chunks[c].begin; p < pl.chunks[c].end; ++p) {
      int32_t ops[2];
      int k = operands(g, pl.order[p], ops);
      for (int j = 0; j < k; ++j) {
        const int32_t u = ops[j];
        if (g.nodes[u].op == XG_OP_INPUT) continue;  // reloaded from the input
        if (chunk_of_node[u] != (int32_t)c) {
          crosses[u] = 1;
          last_phase[u] = std::max(last_phase[u], pl.chunk_phase[c]);
        }
      }
    }
  std::vector<std::vector<int32_t>> release(pl.n_phases + 1);
  std::vector<int32_t> freel;
  int32_t cur = -1;
  struct Occ { int32_t def, last; };
  std::vector<std::vector<Occ>> occupants;
  for (size_t c = 0; c < pl.chunks.size(); ++c) {
    const int32_t ph = pl.chunk_phase[c];
    if (ph != cur) {
      for (int32_t q = std::max(0, cur); q < ph; ++q) {
        for (int32_t sl : release[q]) freel.push_back(sl);
        release[q].clear();
      }
      cur = ph;
    }
    for (int32_t p = pl.chunks[c].begin; p < pl.chunks[c].end; ++p) {
      const int32_t v = pl.order[p];
      if (!crosses[v]) continue;
      int32_t sl;
      if (!freel.empty()) { sl = freel.back(); freel.pop_back(); }
      else sl = pl.n_ws++;
      pl.ws_slot[v] = sl;
      release[last_phase[v]].push_back(sl);
      if ((int32_t)occupants.size() <= sl) occupants.resize(sl + 1);
      occupants[sl].push_back({ph, last_phase[v]});
    }
  }
  // self-check of the invariants the kernel's barriers rely on: an operand
  // comes from the same chunk (earlier), from the inputs, or from the
  // workspace written in an earlier phase; a slot's occupants never overlap
  for (size_t c = 0; c < pl.chunks.size(); ++c)
    for (int32_t p = pl.chunks[c].begin; p < pl.chunks[c].end; ++p) {
      int32_t ops[2];
      int k = operands(g, pl.order[p], ops);
      for (int j = 0; j < k; ++j) {
        const int32_t u = ops[j];
        if (g.nodes[u].op == XG_OP_INPUT) continue;
        const int32_t cu = chunk_of_node[u];
        const bool ok = cu == (int32_t)c ||
                        (pl.ws_slot[u] >= 0 && pl.chunk_phase[cu] < pl.chunk_phase[c]);
        if (!ok) throw std::logic_error("cooperative plan: operand not available");
      }
    }
  for (auto& occ : occupants)
    for (size_t i = 1; i < occ.size(); ++i)
      if (occ[i].def <= occ[i - 1].last) throw std::logic_error("cooperative plan: slot reused too early");
  return pl;
}

Plan make_plan(const Graph& g, const PlanOptions& po) {
  if (po.waves > 1) return make_wide_plan(g, po);
  Plan pl;
  std::vector<int32_t> o1 = original_order(g);
  std::vector<int32_t> o2 = greedy_order(g);
  int64_t m1 = max_live_of(g, o1), m2 = max_live_of(g, o2);
  if (o2.size() == o1.size() && m2 < m1) { pl.order.swap(o2); pl.max_live = m2; }
  else { pl.order.swap(o1); pl.max_live = m1; }
  const int32_t n = (int32_t)g.nodes.size();
  const int32_t L = (int32_t)pl.order.size();
  for (int32_t v : pl.order) if (is_arith(g.nodes[v].op)) pl.n_ops++;

  // live count after each position (for choosing cheap cut points)
  std::vector<int32_t> last(n, -1), pos(n, -1);
  for (int32_t p = 0; p < L; ++p) {
    pos[pl.order[p]] = p;
    int32_t ops[2];
    int k = operands(g, pl.order[p], ops);
    for (int j = 0; j < k; ++j) last[ops[j]] = p;
  }
  std::vector<int32_t> live_after(L, 0);
  {
    std::vector<int32_t> ends(L + 1, 0);
    int32_t live = 0;
    for (int32_t p = 0; p < L; ++p) {
      int32_t v = pl.order[p];
      if (last[v] > p && g.nodes[v].op != XG_OP_INPUT) { live++; ends[last[v]]++; }
      live -= ends[p];
      live_after[p] = live;
    }
  }
  // chunk boundaries: at most chunk_ops operations each, cut where the
  // fewest (non-input) values are live in the last quarter of the window
  const int32_t C = po.chunk_ops > 0 ? po.chunk_ops : INT32_MAX;
  int32_t start = 0;
  while (start < L) {
    if ((int64_t)L - start <= C) { pl.chunks.push_back({start, L}); break; }
    int32_t lo = start + std::max(1, (C * 3) / 4), hi = std::min(L, start + C);
    int32_t best = hi, bl = INT32_MAX;
    for (int32_t p = lo; p <= hi; ++p) {
      if (live_after[p - 1] < bl) { bl = live_after[p - 1]; best = p; }
    }
    pl.chunks.push_back({start, best});
    start = best;
  }
  if (pl.chunks.empty()) pl.chunks.push_back({0, 0});
  // cross-chunk values -> workspace slots (interval colouring over chunks)
  pl.ws_slot.assign(n, -1);
  if (pl.chunks.size() > 1) {
    std::vector<int32_t> chunk_of(L);
    for (int32_t c = 0; c < (int32_t)pl.chunks.size(); ++c)
      for (int32_t p = pl.chunks[c].begin; p < pl.chunks[c].end; ++p) chunk_of[p] = c;
    // last chunk using each value
    std::vector<int32_t> last_chunk(n, -1);
    for (int32_t p = 0; p < L; ++p) {
      int32_t ops[2];
      int k = operands(g, pl.order[p], ops);
      for (int j = 0; j < k; ++j) last_chunk[ops[j]] = std::max(last_chunk[ops[j]], chunk_of[p]);
    }
    // free-slot pool, released when the last reading chunk has passed
    std::vector<std::vector<int32_t>> release((int32_t)pl.chunks.size() + 1);
    std::vector<int32_t> freel;
    int32_t cur_chunk = -1;
    for (int32_t p = 0; p < L; ++p) {
      int32_t c = chunk_of[p];
      if (c != cur_chunk) {
        // slots whose last reader was an earlier chunk become free now
        for (int32_t cc = std::max(0, cur_chunk); cc < c; ++cc) {
          for (int32_t s : release[cc]) freel.push_back(s);
          release[cc].clear();
        }
        cur_chunk = c;
      }
      int32_t v = pl.order[p];
      if (g.nodes[v].op == XG_OP_INPUT) continue;  // reloaded from the input
      if (last_chunk[v] > c) {
        int32_t s;
        if (!freel.empty()) { s = freel.back(); freel.pop_back(); }
        else s = pl.n_ws++;
        pl.ws_slot[v] = s;
        release[last_chunk[v]].push_back(s);
      }
    }
  }
  return pl;
}

}  // namespace xg
