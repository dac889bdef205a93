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

// Phased cooperative-tile plan for narrow graphs (few operations per
// dependency level, where a barrier per level costs more than it gains).
//
// Every value with a single consumer joins its consumer's cluster, so
// clusters are in-trees (a reduction tree stays whole) whose only outside
// operands are inputs, constants and values with several consumers (the
// roots of other clusters).  Clusters costing at most `dup` units (a
// product or sum shared by many trees) are not exchanged: every wave that
// needs one computes its own copy.  The other clusters are list-scheduled
// phase by phase: in each phase every wave takes ready clusters until it
// holds `coop_phase` cost units, a cluster being ready on a wave when each
// value it needs (through its duplicated operands too) was computed in an
// earlier phase or earlier on that wave.  A wave prefers clusters whose
// operands it computed itself (fewer exchanged values), then the longest
// remaining path.  A value read by a wave other than its own goes through
// an LDS exchange slot: written when computed, copied by each reading wave
// right after the barrier that ends its phase (a slot lives for one
// barrier); values stay in their wave's registers otherwise.
namespace {

struct PhasedResult {
  std::vector<std::vector<int32_t>> lists;    // per wave: node ids in order
  std::vector<std::vector<int32_t>> phases;   // per wave: phase of each list entry
  std::vector<int32_t> node_phase;            // non-duplicated nodes: their phase
  std::vector<int32_t> owner;                 // non-duplicated nodes: their wave (-1: duplicated)
  int32_t n_phases = 0;
  int64_t est = 0;                            // modelled time (cost units)
};

PhasedResult phased_schedule(const Graph& g, int W, int64_t T, int64_t dup_max, int64_t cut_max) {
  const int32_t n = (int32_t)g.nodes.size();
  auto sched = [&](int32_t v) {
    const int op = g.nodes[v].op;
    return op != XG_OP_CONST && op != XG_OP_INPUT;
  };
  std::vector<int32_t> nuse(n, 0), single(n, -1);
  std::vector<char> is_out(n, 0);
  for (auto& a : g.out) for (int32_t v : a) is_out[v] = 1;
  for (int32_t v = 0; v < n; ++v) {
    if (!sched(v)) continue;
    int32_t ops[2];
    int k = operands(g, v, ops);
    for (int j = 0; j < k; ++j) { nuse[ops[j]]++; single[ops[j]] = v; }
  }
  // A single-consumer subtree stops growing at about cut_max cost units:
  // its top becomes a cluster of its own, so a large independent subtree
  // (a sum of many products) is not bundled with a consumer that must wait
  // for other values (a triangular-solve step), and waves can share it
  std::vector<int64_t> tree(n, 0);
  std::vector<char> cut(n, 0);
  for (int32_t v = 0; v < n; ++v) {
    if (!sched(v)) continue;
    int32_t ops[2];
    int k = operands(g, v, ops);
    int64_t t = op_cost(g.nodes[v].op);
    for (int j = 0; j < k; ++j)
      if (sched(ops[j]) && nuse[ops[j]] == 1 && !cut[ops[j]]) t += tree[ops[j]];
    tree[v] = t;
    if (nuse[v] == 1 && cut_max > 0 && t >= cut_max) cut[v] = 1;
  }
  std::vector<int32_t> root(n, -1);
  for (int32_t v = n - 1; v >= 0; --v)
    if (sched(v)) root[v] = (nuse[v] == 1 && !cut[v]) ? root[single[v]] : v;
  std::vector<std::vector<int32_t>> members(n);
  for (int32_t v = 0; v < n; ++v)
    if (sched(v)) members[root[v]].push_back(v);  // increasing ids: topological
  std::vector<int32_t> clusters;
  std::vector<int64_t> ccost(n, 0);
  std::vector<std::vector<int32_t>> cpred(n);
  std::vector<char> dup(n, 0);
  for (int32_t r = 0; r < n; ++r) {
    if (members[r].empty()) continue;
    clusters.push_back(r);
    bool has_out = false;
    for (int32_t v : members[r]) {
      ccost[r] += op_cost(g.nodes[v].op);
      has_out = has_out || is_out[v];
      int32_t ops[2];
      int k = operands(g, v, ops);
      for (int j = 0; j < k; ++j) {
        const int32_t u = ops[j];
        if (g.nodes[u].op == XG_OP_INPUT || root[u] == r) continue;
        cpred[r].push_back(root[u]);
      }
    }
    std::sort(cpred[r].begin(), cpred[r].end());
    cpred[r].erase(std::unique(cpred[r].begin(), cpred[r].end()), cpred[r].end());
    dup[r] = ccost[r] <= dup_max && !has_out && nuse[r] > 0;
  }
  // effective predecessors (exchanged clusters reached through duplicated
  // ones) and the duplicated clusters each cluster pulls in, in order
  std::vector<std::vector<int32_t>> eff(n), cone(n);
  for (int32_t r : clusters) {
    std::vector<int32_t> e, d;
    for (int32_t p : cpred[r]) {
      if (dup[p]) {
        e.insert(e.end(), eff[p].begin(), eff[p].end());
        d.insert(d.end(), cone[p].begin(), cone[p].end());
        d.push_back(p);
      } else {
        e.push_back(p);
      }
    }
    std::sort(e.begin(), e.end());
    e.erase(std::unique(e.begin(), e.end()), e.end());
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    eff[r].swap(e);
    cone[r].swap(d);
  }
  std::vector<int32_t> sc;  // scheduled (exchanged) clusters
  std::vector<std::vector<int32_t>> esucc(n);
  for (int32_t r : clusters)
    if (!dup[r]) {
      sc.push_back(r);
      for (int32_t p : eff[r]) esucc[p].push_back(r);
    }
  std::vector<int64_t> bl(n, 0);
  for (auto it = sc.rbegin(); it != sc.rend(); ++it) {
    int64_t m = 0;
    for (int32_t s : esucc[*it]) m = std::max(m, bl[s]);
    bl[*it] = ccost[*it] + m;
  }
  struct Key {
    int32_t local;
    int64_t bl;
    int32_t r;
    bool operator<(const Key& o) const {  // max-heap: more local, longer path, smaller id
      if (local != o.local) return local < o.local;
      if (bl != o.bl) return bl < o.bl;
      return r > o.r;
    }
  };
  std::vector<std::priority_queue<Key>> ready(W);
  std::vector<std::vector<int32_t>> miss(W, std::vector<int32_t>(n, 0)), nloc(W, std::vector<int32_t>(n, 0));
  std::vector<std::vector<char>> have(W, std::vector<char>(n, 0));  // duplicated clusters on each wave
  for (int w = 0; w < W; ++w)
    for (int32_t r : sc) {
      miss[w][r] = (int32_t)eff[r].size();
      if (miss[w][r] == 0) ready[w].push({0, bl[r], r});
    }
  PhasedResult res;
  res.lists.assign(W, {});
  res.phases.assign(W, {});
  res.node_phase.assign(n, -1);
  res.owner.assign(n, -1);
  std::vector<char> done(n, 0);
  std::vector<int32_t> cphase(n, -1), cwave(n, -1);
  size_t remaining = sc.size();
  int32_t phase = 0;
  std::vector<std::vector<int64_t>> loads;
  while (remaining > 0) {
    std::vector<int64_t> load(W, 0);
    std::vector<std::pair<int, int32_t>> newly;
    std::vector<char> active(W, 1);
    int n_active = W;
    bool starved = false;  // a wave found nothing ready in this phase
    while (n_active > 0) {
      int w = -1;
      for (int x = 0; x < W; ++x)
        if (active[x] && (w < 0 || load[x] < load[w])) w = x;
      auto& q = ready[w];
      while (!q.empty() && done[q.top().r]) q.pop();
      // a phase lasts at least T; once a wave took a large cluster, the
      // others fill up to its load (they would wait at the barrier anyway).
      // While some wave has nothing to do, the phase is cut short instead:
      // the busy waves' new values reach the idle ones at the next barrier
      int64_t target = T;
      for (int x = 0; x < W; ++x) target = std::max(target, load[x]);
      if (starved) target = std::max<int64_t>(40, T / 4);
      if (q.empty() || load[w] >= target) {
        if (q.empty()) starved = true;
        active[w] = 0;
        --n_active;
        continue;
      }
      const int32_t r = q.top().r;
      q.pop();
      done[r] = 1;
      --remaining;
      for (int32_t d : cone[r]) {
        if (have[w][d]) continue;
        have[w][d] = 1;
        load[w] += ccost[d];
        for (int32_t v : members[d]) { res.lists[w].push_back(v); res.phases[w].push_back(phase); }
      }
      load[w] += ccost[r];
      for (int32_t v : members[r]) {
        res.lists[w].push_back(v);
        res.phases[w].push_back(phase);
        res.node_phase[v] = phase;
        res.owner[v] = w;
      }
      cphase[r] = phase;
      cwave[r] = w;
      newly.push_back({w, r});
      for (int32_t s : esucc[r]) {
        nloc[w][s]++;
        if (--miss[w][s] == 0 && !done[s]) ready[w].push({nloc[w][s], bl[s], s});
      }
    }
    if (newly.empty()) throw std::logic_error("phased plan: no cluster became ready");
    for (auto& wr : newly)
      for (int x = 0; x < W; ++x) {
        if (x == wr.first) continue;
        for (int32_t s : esucc[wr.second])
          if (--miss[x][s] == 0 && !done[s]) ready[x].push({nloc[x][s], bl[s], s});
      }
    loads.push_back(load);
    ++phase;
  }
  res.n_phases = phase;
  // modelled time: per phase the slowest wave, each exchanged value costing
  // its producer a store and each reading wave a load, plus a barrier
  std::vector<std::vector<int64_t>> xfer(phase + 1, std::vector<int64_t>(W, 0));
  for (int w = 0; w < W; ++w) {
    std::vector<char> got(n, 0);
    for (int32_t v : res.lists[w]) {
      int32_t ops[2];
      int k = operands(g, v, ops);
      for (int j = 0; j < k; ++j) {
        const int32_t u = ops[j];
        if (g.nodes[u].op == XG_OP_INPUT || res.owner[u] < 0 || res.owner[u] == w || got[u]) continue;
        got[u] = 1;
        xfer[res.node_phase[u] + 1][w] += 1;
        xfer[res.node_phase[u]][res.owner[u]] += 1;
      }
    }
  }
  res.est = 0;
  for (int32_t k = 0; k < phase; ++k) {
    int64_t m = 0;
    for (int w = 0; w < W; ++w) m = std::max(m, loads[k][w] + xfer[k][w]);
    res.est += m + 30;
  }
  return res;
}

}  // namespace

static Plan make_phased_plan(const Graph& g, const PlanOptions& po) {
  const int32_t n = (int32_t)g.nodes.size();
  const int W = po.waves;
  const int64_t T = std::max(1, po.coop_phase);
  // duplicate clusters of up to 1, 2, 4 or 8 cost units: the plan with the
  // best modelled time among those whose exchange fits the LDS allowance
  Plan best;
  int64_t best_est = INT64_MAX;
  bool best_lds_only = false;
  std::string why = "phased plan: no duplication threshold fits the LDS";
  for (int64_t D : {1, 2, 4, 8})
  for (int64_t S : {0, 32, 96}) {
    PhasedResult r = phased_schedule(g, W, T, D, S);
    Plan pl;
    pl.waves = W;
    pl.phased = true;
    pl.n_phases = r.n_phases;
    pl.node_phase = r.node_phase;
    // schedule: wave 0's nodes, then wave 1's, ...; one chunk per wave
    for (int w = 0; w < W; ++w) {
      const int32_t begin = (int32_t)pl.order.size();
      if (w == 0)  // inputs that are outputs themselves are stored by wave 0
        for (int32_t v = 0; v < n; ++v)
          if (g.nodes[v].op == XG_OP_INPUT) { pl.order.push_back(v); pl.pos_phase.push_back(0); }
      for (size_t i = 0; i < r.lists[w].size(); ++i) {
        pl.order.push_back(r.lists[w][i]);
        pl.pos_phase.push_back(r.phases[w][i]);
      }
      pl.chunks.push_back({begin, (int32_t)pl.order.size()});
      pl.chunk_wave.push_back(w);
      pl.chunk_phase.push_back(0);
    }
    for (int32_t v = 0; v < n; ++v)
      if (is_arith(g.nodes[v].op)) pl.n_ops++;
    for (auto& ch : pl.chunks) {
      std::vector<int32_t> part(pl.order.begin() + ch.begin, pl.order.begin() + ch.end);
      pl.max_live = std::max(pl.max_live, max_live_of(g, part));
    }
    // exchange slots (values other waves read) and each wave's mailbox
    pl.ws_slot.assign(n, -1);
    pl.xch_slot.assign(n, -1);
    pl.mailbox.assign((size_t)W * (pl.n_phases + 1), {});
    std::vector<char> remote(n, 0);
    for (int w = 0; w < W; ++w) {
      std::vector<char> got(n, 0);
      const Chunk& ch = pl.chunks[w];
      for (int32_t p = ch.begin; p < ch.end; ++p) {
        const int32_t v = pl.order[p];
        if (g.nodes[v].op == XG_OP_INPUT) continue;
        int32_t ops[2];
        int k = operands(g, v, ops);
        for (int j = 0; j < k; ++j) {
          const int32_t u = ops[j];
          if (g.nodes[u].op == XG_OP_INPUT || r.owner[u] < 0 || r.owner[u] == w || got[u]) continue;
          got[u] = 1;
          remote[u] = 1;
          pl.mailbox[(size_t)w * (pl.n_phases + 1) + r.node_phase[u] + 1].push_back(u);
        }
      }
    }
    // values of phase k are copied in phase k + 1; their slots are reused
    // by values of phase k + 2 on
    std::vector<std::vector<int32_t>> by_phase(pl.n_phases);
    for (int32_t v = 0; v < n; ++v)
      if (remote[v]) by_phase[r.node_phase[v]].push_back(v);
    // LDS slots up to the allowance, then workspace slots (the same
    // one-barrier lifetime; a workspace copy is reloaded only by the
    // mailbox, each wave then keeps its own)
    std::vector<int32_t> freel, freew;
    const int64_t cap = po.xch_cap > 0 ? po.xch_cap : INT64_MAX;
    int64_t ws_loads = 0;
    for (int32_t ph = 0; ph < pl.n_phases; ++ph) {
      if (ph >= 2)
        for (int32_t v : by_phase[ph - 2]) {
          if (pl.xch_slot[v] >= 0) freel.push_back(pl.xch_slot[v]);
          else freew.push_back(pl.ws_slot[v]);
        }
      for (int32_t v : by_phase[ph]) {
        if (!freel.empty()) { pl.xch_slot[v] = freel.back(); freel.pop_back(); }
        else if (pl.n_xch < cap) pl.xch_slot[v] = pl.n_xch++;
        else if (!freew.empty()) { pl.ws_slot[v] = freew.back(); freew.pop_back(); }
        else pl.ws_slot[v] = pl.n_ws++;
      }
    }
    for (auto& mb : pl.mailbox)
      for (int32_t u : mb) ws_loads += pl.ws_slot[u] >= 0;
    // a workspace exchange costs its reader a global load (L2 latency),
    // far more than an LDS one
    r.est += 8 * ws_loads / W;
    // self-check: an operand is an input, computed earlier on the same wave,
    // or computed by another wave in an earlier phase and exchanged; phases
    // never decrease along a wave's list
    for (auto& ch : pl.chunks) {
      std::vector<char> seen(n, 0);
      for (int32_t p = ch.begin; p < ch.end; ++p) {
        const int32_t v = pl.order[p];
        if (g.nodes[v].op != XG_OP_INPUT) {
          int32_t ops[2];
          int k = operands(g, v, ops);
          for (int j = 0; j < k; ++j) {
            const int32_t u = ops[j];
            if (g.nodes[u].op == XG_OP_INPUT || seen[u]) continue;
            if (!((pl.xch_slot[u] >= 0 || pl.ws_slot[u] >= 0) && r.node_phase[u] < pl.pos_phase[p]))
              throw std::logic_error("phased plan: operand not available");
          }
          if (p > ch.begin && pl.pos_phase[p] < pl.pos_phase[p - 1])
            throw std::logic_error("phased plan: phases out of order");
        }
        seen[v] = 1;
      }
    }
    // plans whose exchanges all fit the LDS come first; workspace
    // exchanges (and the spills that come with such wide plans) are only
    // taken when no plan fits
    const bool lds_only = pl.n_ws == 0;
    if (lds_only && (!best_lds_only || r.est < best_est)) {
      best_est = r.est;
      best_lds_only = true;
      pl.coop_est = r.est;
      best = std::move(pl);
    } else if (!lds_only && !best_lds_only && r.est < best_est) {
      best_est = r.est;
      pl.coop_est = r.est;
      best = std::move(pl);
    }
  }
  if (best_est == INT64_MAX) throw std::logic_error(why);
  return best;
}

Plan make_plan(const Graph& g, const PlanOptions& po) {
  if (po.waves > 1 && po.coop_phase > 0) return make_phased_plan(g, po);
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
