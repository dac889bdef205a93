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

Plan make_plan(const Graph& g, const PlanOptions& po) {
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
