// Host planner (see plan.hpp).
//
// Elimination lists follow Sec. 3.1 / Sec. 3.2 of the paper (FlatTree ==
// Sameh-Kuck, BinaryTree, Fibonacci, PlasmaTree, and the run-time pairings
// ASAP and GRASAP(k) of the tiled model) and Algorithm 4 (Greedy).
// The expansion into kernels follows Algorithms 2 (TS) and 3 (TT), skipping
// GEQRT on tiles that are already triangles (Sec. 2.1).  The schedule is the
// unbounded-processor as-soon-as-possible execution of Sec. 2.3 with the
// Table 1 weights.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <queue>
#include <set>
#include <tuple>

namespace tqr {

bool valid_shape(int p, int q, int tree, int bs) {
  if (q < 1 || p < q) return false;
  if (tree < T_FLAT || tree > T_HADRI) return false;
  if ((tree == T_PLASMA || tree == T_HADRI) && (bs < 1 || bs > p)) return false;
  if (tree == T_GRASAP && (bs < 0 || bs > q)) return false;
  return true;
}

int resolve_family(int tree, int family) {
  if (family == F_DEFAULT) return tree == T_FLAT ? F_TS : F_TT;
  return family;
}

namespace {

// Smallest t >= 0 with t(t+1)/2 >= v.
int tri_ceil(int v) {
  int t = 0;
  while (t * (t + 1) / 2 < v) ++t;
  return t;
}

void flat(int p, int q, std::vector<Elim>& out) {
  const int kmax = std::min(p, q);
  for (int k = 1; k <= kmax; ++k)
    for (int i = k + 1; i <= p; ++i) out.push_back({i, k, k});
}

// Binary reduction over rows k..p of each column, rooted at row k.
void binary(int p, int q, std::vector<Elim>& out) {
  const int kmax = std::min(p, q);
  for (int k = 1; k <= kmax; ++k) {
    const int rows = p - k + 1;
    for (int stride = 1; stride < rows; stride <<= 1)
      for (int off = stride; off < rows; off += 2 * stride)
        out.push_back({k + off, k + off - stride, k});
  }
}

// Fibonacci (Modi-Clarke order 1): tile (i, k) is zeroed at step
// x - y(i - k + 1) + 1 + 2(k - 1), x minimal with x(x+1)/2 >= p - 1 and
// y(r) minimal with r <= y(y+1)/2 + 1.  Tiles zeroed at one step form a run
// of z consecutive rows paired with the z rows just above them.
void fibonacci(int p, int q, std::vector<Elim>& out) {
  const int x = tri_ceil(p - 1);
  const int kmax = std::min(p, q);
  std::vector<int> step(p + 2, 0);
  for (int k = 1; k <= kmax; ++k) {
    int smin = 1 << 30, smax = -1;
    for (int i = k + 1; i <= p; ++i) {
      const int y = tri_ceil(i - k);  // least y with i-k+1 <= y(y+1)/2 + 1
      step[i] = x - y + 1 + 2 * (k - 1);
      smin = std::min(smin, step[i]);
      smax = std::max(smax, step[i]);
    }
    for (int s = smin; s <= smax; ++s) {
      int first = -1, z = 0;
      for (int i = k + 1; i <= p; ++i)
        if (step[i] == s) {
          if (first < 0) first = i;
          ++z;
        }
      for (int t = 0; t < z; ++t) out.push_back({first + t, first + t - z, k});
    }
  }
}

// Greedy, Algorithm 4: rounds over columns q..1 with counters nT(j) of
// triangularized and nZ(j) of zeroed tiles.
void greedy(int p, int q, std::vector<Elim>& out) {
  std::vector<int> nT(q + 1, 0), nZ(q + 1, 0);
  auto done = [&] { return nZ[q] == p - q && nT[q] == p - q + 1; };
  while (!done()) {
    for (int j = q; j >= 1; --j) {
      const int tri_next = (j == 1) ? p : nZ[j - 1];
      const int zero_next = nZ[j] + (nT[j] - nZ[j]) / 2;
      const int shift = zero_next - nZ[j];
      for (int kk = nZ[j]; kk < zero_next; ++kk) out.push_back({p - kk, p - kk - shift, j});
      nT[j] = tri_next;
      nZ[j] = zero_next;
    }
  }
}

// PlasmaTree(BS): domains of BS rows starting at row k; flat inside each
// domain, then a binary tree over the domain heads.
void plasma(int p, int q, int bs, std::vector<Elim>& out) {
  const int kmax = std::min(p, q);
  std::vector<int> heads;
  for (int k = 1; k <= kmax; ++k) {
    heads.clear();
    for (int h = k; h <= p; h += bs) heads.push_back(h);
    for (int h : heads)
      for (int i = h + 1; i <= std::min(h + bs - 1, p); ++i) out.push_back({i, h, k});
    const int nd = static_cast<int>(heads.size());
    for (int stride = 1; stride < nd; stride <<= 1)
      for (int d = stride; d < nd; d += 2 * stride) out.push_back({heads[d], heads[d - stride], k});
  }
}

// Hadri et al.'s Semi-Parallel (TS) / Fully-Parallel (TT) tile CAQR trees as
// Sec. 4 describes them: PlasmaTree's flat domains of BS rows and binary
// merge of the domain heads, but with the domains fixed at rows 1..BS,
// BS+1..2BS, ..., so the top domain shrinks as the columns advance.
void hadri(int p, int q, int bs, std::vector<Elim>& out) {
  const int kmax = std::min(p, q);
  std::vector<int> heads;
  for (int k = 1; k <= kmax; ++k) {
    heads.assign(1, k);
    for (int h = bs + 1; h <= p; h += bs)
      if (h > k) heads.push_back(h);
    const int nd = static_cast<int>(heads.size());
    for (int d = 0; d < nd; ++d) {
      const int end = (d + 1 < nd) ? heads[d + 1] - 1 : p;
      for (int i = heads[d] + 1; i <= end; ++i) out.push_back({i, heads[d], k});
    }
    for (int stride = 1; stride < nd; stride <<= 1)
      for (int d = stride; d < nd; d += 2 * stride) out.push_back({heads[d], heads[d - stride], k});
  }
}

// ASAP and GRASAP(kdyn), Sec. 3.2 (Table 4): the pairs of the last kdyn
// columns (all of them for ASAP) are chosen while a unit-weight execution
// with TT kernels and the Table 1 weights runs; the columns before them take
// the Greedy pairs in Greedy's order.  A row is ready in column k once
// GEQRT(i, k) has finished (after every update of tile (i, k) from column
// k - 1) and idle when no TTQRT that uses it is running.  At each time at
// which a row of a run-time column becomes ready or idle, the r ready idle
// rows of that column (top to bottom) are paired: the bottom s = r / 2 are
// killed by the s rows right above them.  Every other task starts when its
// inputs are ready (Algorithm 3's data flow: GEQRT and UNMQR after the last
// update of their tiles, TTMQR after its TTQRT and both tiles' last
// updates; a TTQRT needs only the two triangles).  The list is the static
// part in order, then the run-time eliminations by start time, column and
// killed row, so the ordinary task expansion schedules it as it ran.
void dynamic_pairs(int p, int q, int kdyn, std::vector<Elim>& out) {
  const int kmax = std::min(p, q);
  const int cut = (kdyn <= 0) ? kmax + 1 : std::max(1, kmax - kdyn + 1);  // first run-time column
  const int64_t WG = kWeight[K_GEQRT], WU = kWeight[K_UNMQR], WQ = kWeight[K_TTQRT], WM = kWeight[K_TTMQR];
  std::vector<int64_t> avail(static_cast<size_t>(p + 1) * (q + 1), 0);  // last update of tile (r, j)
  std::vector<int64_t> ready(static_cast<size_t>(p + 1) * (kmax + 2), -1);  // GEQRT(r, k) finish
  std::vector<int64_t> busy(p + 1, 0);                                       // running TTQRT finish
  auto A = [&](int r, int j) -> int64_t& { return avail[static_cast<size_t>(r) * (q + 1) + j]; };
  auto R = [&](int r, int k) -> int64_t& { return ready[static_cast<size_t>(r) * (kmax + 2) + k]; };
  auto enter = [&](int r, int k) {
    const int64_t f = A(r, k) + WG;
    R(r, k) = f;
    A(r, k) = f;
    for (int j = k + 1; j <= q; ++j) A(r, j) = std::max(f, A(r, j)) + WU;
    return f;
  };
  // TTQRT(i, piv, k) at t with its updates; returns row i's GEQRT finish in
  // column k + 1, or -1.
  auto eliminate = [&](int i, int piv, int k, int64_t t) -> int64_t {
    const int64_t f = t + WQ;
    busy[i] = busy[piv] = f;
    for (int j = k + 1; j <= q; ++j) {
      const int64_t u = std::max(f, std::max(A(piv, j), A(i, j))) + WM;
      A(piv, j) = A(i, j) = u;
    }
    return (k + 1 <= kmax) ? enter(i, k + 1) : -1;
  };
  for (int r = 1; r <= p; ++r) enter(r, 1);
  if (cut > 1) {
    std::vector<Elim> g;
    greedy(p, q, g);
    std::vector<int64_t> tri(static_cast<size_t>(p + 1) * (kmax + 2), 0);  // triangle free
    auto T = [&](int r, int k) -> int64_t& { return tri[static_cast<size_t>(r) * (kmax + 2) + k]; };
    for (int r = 1; r <= p; ++r) T(r, 1) = R(r, 1);
    for (const Elim& e : g) {
      if (e.k >= cut) continue;
      const int64_t t = std::max(T(e.piv, e.k), T(e.i, e.k));
      const int64_t f = eliminate(e.i, e.piv, e.k, t);
      T(e.piv, e.k) = t + WQ;
      if (f >= 0) T(e.i, e.k + 1) = f;
      out.push_back(e);
    }
  }
  // Run-time columns, event by event (time, column).
  std::vector<std::set<int>> alive(kmax + 2);
  std::priority_queue<std::pair<int64_t, int>, std::vector<std::pair<int64_t, int>>, std::greater<>> ev;
  for (int k = cut; k <= kmax; ++k)
    for (int r = k; r <= p; ++r)
      if (R(r, k) >= 0) {
        alive[k].insert(r);
        ev.push({R(r, k), k});
      }
  struct Dyn { int64_t t; int k, i, piv; };
  std::vector<Dyn> dyn;
  std::vector<int> rows;
  while (!ev.empty()) {
    const int64_t t = ev.top().first;
    std::set<int> cols;
    while (!ev.empty() && ev.top().first == t) {
      cols.insert(ev.top().second);
      ev.pop();
    }
    for (int k : cols) {
      rows.clear();
      for (int r : alive[k])
        if (R(r, k) <= t && busy[r] <= t) rows.push_back(r);
      const int s = static_cast<int>(rows.size()) / 2;
      if (s == 0) continue;
      const int n = static_cast<int>(rows.size());
      for (int a = 0; a < s; ++a) {
        const int piv = rows[n - 2 * s + a], i = rows[n - s + a];
        const int64_t f = eliminate(i, piv, k, t);
        alive[k].erase(i);
        dyn.push_back({t, k, i, piv});
        if (f >= 0) {
          alive[k + 1].insert(i);
          ev.push({f, k + 1});
        }
      }
      ev.push({t + WQ, k});
    }
  }
  std::sort(dyn.begin(), dyn.end(), [](const Dyn& a, const Dyn& b) {
    return std::tie(a.t, a.k, a.i, a.piv) < std::tie(b.t, b.k, b.i, b.piv);
  });
  for (const Dyn& d : dyn) out.push_back({d.i, d.piv, d.k});
}

}  // namespace

bool make_elims(int p, int q, int tree, int bs, std::vector<Elim>& out) {
  out.clear();
  if (!valid_shape(p, q, tree, bs)) return false;
  switch (tree) {
    case T_FLAT:
    case T_SAMEH_KUCK: flat(p, q, out); break;
    case T_BINARY: binary(p, q, out); break;
    case T_FIBONACCI: fibonacci(p, q, out); break;
    case T_GREEDY: greedy(p, q, out); break;
    case T_PLASMA: plasma(p, q, bs, out); break;
    case T_ASAP: dynamic_pairs(p, q, std::min(p, q), out); break;
    case T_GRASAP: dynamic_pairs(p, q, bs, out); break;
    case T_HADRI: hadri(p, q, bs, out); break;
    default: return false;
  }
  return true;
}

namespace {

// Task expansion with tile data flow.  For every tile we remember the last
// task that wrote its "upper" part (R, or the TT reflectors, or the whole
// tile while it is full) and its "lower" part (GEQRT reflectors).
struct Expander {
  int p, q, family;
  std::vector<Task>& tasks;
  std::vector<std::vector<int32_t>> preds;
  std::vector<int32_t> up, lo;
  std::vector<char> is_tri;

  Expander(int p_, int q_, int fam, std::vector<Task>& t)
      : p(p_), q(q_), family(fam), tasks(t),
        up(static_cast<size_t>(p_) * q_, -1), lo(static_cast<size_t>(p_) * q_, -1),
        is_tri(static_cast<size_t>(p_) * q_, 0) {}

  size_t at(int r, int c) const { return static_cast<size_t>(r - 1) * q + (c - 1); }

  int emit(Task t, std::initializer_list<int32_t> d) {
    std::vector<int32_t> v;
    for (int32_t x : d)
      if (x >= 0) v.push_back(x);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    tasks.push_back(t);
    preds.push_back(std::move(v));
    return static_cast<int>(tasks.size()) - 1;
  }

  void factor_row(int r, int k) {
    const size_t a = at(r, k);
    const int g = emit({K_GEQRT, r, 0, k, 0}, {up[a], lo[a]});
    up[a] = lo[a] = g;
    is_tri[a] = 1;
    for (int j = k + 1; j <= q; ++j) {
      const size_t c = at(r, j);
      const int u = emit({K_UNMQR, r, 0, k, j}, {g, up[c], lo[c]});
      up[c] = lo[c] = u;
    }
  }

  void run(const std::vector<Elim>& el) {
    // Rows acting as a pivot in each column (to find the leaves for TS).
    std::vector<char> pivot(static_cast<size_t>(p + 1) * (q + 1), 0);
    for (const Elim& e : el) pivot[static_cast<size_t>(e.k) * (p + 1) + e.piv] = 1;
    for (const Elim& e : el) {
      const int i = e.i, pv = e.piv, k = e.k;
      if (!is_tri[at(pv, k)]) factor_row(pv, k);
      const bool leaf = !pivot[static_cast<size_t>(k) * (p + 1) + i];
      const size_t ti = at(i, k), tp = at(pv, k);
      int f, upd;
      if (family == F_TS && leaf && !is_tri[ti]) {
        f = emit({K_TSQRT, i, pv, k, 0}, {up[tp], up[ti], lo[ti]});
        up[tp] = f;
        up[ti] = lo[ti] = f;
        upd = K_TSMQR;
      } else {
        if (!is_tri[ti]) factor_row(i, k);
        f = emit({K_TTQRT, i, pv, k, 0}, {up[tp], up[ti]});
        up[tp] = f;
        up[ti] = f;
        upd = K_TTMQR;
      }
      for (int j = k + 1; j <= q; ++j) {
        const size_t cp = at(pv, j), ci = at(i, j);
        const int u = emit({upd, i, pv, k, j}, {f, up[cp], lo[cp], up[ci], lo[ci]});
        up[cp] = lo[cp] = up[ci] = lo[ci] = u;
      }
    }
    if (p == q && !is_tri[at(q, q)]) factor_row(q, q);
  }
};

}  // namespace

bool make_plan(int p, int q, int tree, int bs, int family, Plan& plan) {
  if (!valid_shape(p, q, tree, bs)) return false;
  family = resolve_family(tree, family);
  if (family != F_TT && family != F_TS) return false;
  plan = Plan();
  plan.p = p;
  plan.q = q;
  plan.tree = tree;
  plan.bs = bs;
  plan.family = family;
  if (!make_elims(p, q, tree, bs, plan.elims)) return false;
  Expander ex(p, q, family, plan.tasks);
  ex.run(plan.elims);
  const size_t n = plan.tasks.size();
  plan.pred_ptr.assign(n + 1, 0);
  for (size_t t = 0; t < n; ++t) plan.pred_ptr[t + 1] = plan.pred_ptr[t] + ex.preds[t].size();
  plan.pred_idx.reserve(plan.pred_ptr[n]);
  for (auto& v : ex.preds) plan.pred_idx.insert(plan.pred_idx.end(), v.begin(), v.end());
  plan.start.assign(n, 0);
  plan.finish.assign(n, 0);
  plan.cp = 0;
  for (size_t t = 0; t < n; ++t) {
    int64_t s = 0;
    for (int64_t e = plan.pred_ptr[t]; e < plan.pred_ptr[t + 1]; ++e)
      s = std::max(s, plan.finish[plan.pred_idx[e]]);
    plan.start[t] = s;
    plan.finish[t] = s + kWeight[plan.tasks[t].kind];
    plan.cp = std::max(plan.cp, plan.finish[t]);
  }
  return true;
}

// Every predecessor of subtask r of an executor plan: the ones waited for
// before it starts, the streamed C1 writer and the streamed panel blocks.
std::vector<int32_t> stream_preds(const ExecPlan& ex, size_t r) {
  const SubTask& st = ex.sub[r];
  std::vector<int32_t> v;
  for (int32_t e = st.dep_begin; e < st.dep_end; ++e) v.push_back(dep_index(ex.deps[e]));
  if (st.sdep >= 0) v.push_back(st.sdep);
  if (st.pdep >= 0)
    for (int b = 0; b < ex.pblk; ++b) v.push_back(dep_index(ex.deps[st.pdep + b]));
  return v;
}

// Start order of a list schedule of the executor subtasks (emission order,
// predecessor entries pre, streamed C1 writer sdep, first streamed panel
// block pfirst) on `workers` workgroups: whenever a workgroup is free it
// starts the ready subtask of largest bottom level bl.  A subtask is ready
// once its plain predecessors have ended, its early ones have released
// (a panel block releases after 0.65 of its weight, the last block of a
// panel task at its end), and its streamed predecessors have started
// (every block of a streamed panel task, so that the dispatch order keeps
// them ahead of the update).  Waits inside a panel block subtask (stages 1
// and 2) pair with early entries for the same predecessors and are not
// start conditions.  Durations are the weights wt.  Returns each subtask's
// rank, a topological order.
static std::vector<double> sim_order(const std::vector<SubTask>& sub, const std::vector<std::vector<int32_t>>& pre,
                                     const std::vector<int32_t>& sdep, const std::vector<int32_t>& pfirst, int pblk,
                                     const std::vector<double>& wt, const std::vector<double>& bl, int workers) {
  const size_t n = sub.size();
  std::vector<int32_t> nwait(n, 0);
  std::vector<std::vector<int32_t>> on_start(n), on_early(n), on_end(n);
  for (size_t s = 0; s < n; ++s) {
    for (int32_t d : pre[s]) {
      if (dep_stage(d) != 0) continue;
      (dep_early(d) ? on_early : on_end)[dep_index(d)].push_back(static_cast<int32_t>(s));
      ++nwait[s];
    }
    if (sdep[s] >= 0) {
      on_start[sdep[s]].push_back(static_cast<int32_t>(s));
      ++nwait[s];
    }
    if (pfirst[s] >= 0)
      for (int b = 0; b < pblk; ++b) {
        on_start[pfirst[s] + b].push_back(static_cast<int32_t>(s));
        ++nwait[s];
      }
  }
  // ready subtasks: largest bottom level first, then emission order
  auto cmp = [&](int32_t a, int32_t b) { return bl[a] != bl[b] ? bl[a] < bl[b] : a > b; };
  std::priority_queue<int32_t, std::vector<int32_t>, decltype(cmp)> ready(cmp);
  // events: (time, kind 0 = early release / 1 = end, subtask), earliest first
  using Ev = std::tuple<double, int, int32_t>;
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> ev;
  auto notify = [&](const std::vector<int32_t>& v) {
    for (int32_t c : v)
      if (--nwait[c] == 0) ready.push(c);
  };
  for (size_t s = 0; s < n; ++s)
    if (nwait[s] == 0) ready.push(static_cast<int32_t>(s));
  std::vector<double> rank(n, 0.0);
  size_t started = 0;
  int free = workers;
  double now = 0.0;
  while (started < n) {
    while (free > 0 && !ready.empty()) {
      const int32_t s = ready.top();
      ready.pop();
      rank[s] = static_cast<double>(started++);
      --free;
      const int kd = sub[s].kind;
      const bool panel_blk = (kd == K_GEQRT || kd == K_TSQRT || kd == K_TTQRT) && sub[s].slab >= 0;
      const double rel = (panel_blk && sub[s].slab < pblk - 1) ? 0.65 : 1.0;
      ev.emplace(now + rel * wt[s], 0, s);
      ev.emplace(now + wt[s], 1, s);
      notify(on_start[s]);
    }
    if (ev.empty()) break;  // cannot happen for a DAG
    now = std::get<0>(ev.top());
    while (!ev.empty() && std::get<0>(ev.top()) <= now) {
      const int kind = std::get<1>(ev.top());
      const int32_t s = std::get<2>(ev.top());
      ev.pop();
      if (kind == 0) {
        notify(on_early[s]);
      } else {
        notify(on_end[s]);
        ++free;
      }
    }
  }
  return rank;
}

// ---------------------------------------------------------------------------
// Executor plan.  An update task on column slab s of its C tiles only touches
// slab s, so dependencies are tracked per (tile, slab); the panel tasks touch
// every slab of their tiles.  The two parts of a tile (upper / lower) are
// tracked separately as in the task expansion.
//
// With pblk > 1 a panel task becomes pblk subtasks, one per inner block b of
// ib columns (c0 = b ib), in order.  Block b of a panel task reads and writes
// only rows c0 .. c0 + ib - 1 of its pivot triangle R1 (TSQRT, TTQRT), rows
// 0 .. c0 + ib - 1 of a killed triangle (TTQRT), and rows c0 .. nb - 1 of a
// tile it triangularizes (GEQRT), each in columns >= c0.  So on a tile that
// an earlier panel task of the same column wrote, block b only has to wait
// for block b of that task (which follows its blocks 0 .. b - 1), not for
// the whole task: consecutive panel tasks on a pivot pipeline block by
// block.  Block 0 waits for the task's other (update) predecessors, block b
// for block b - 1, and later tasks depend on the last block.
//
// With stream, two kinds of edges are streamed: the subtask starts without
// waiting for the predecessor to finish and follows it block by block
// inside the kernel.
//   pdep: an update subtask applies the ib-blocks of reflectors of one panel
//   task in order, and block b only needs panel block b (its reflectors and
//   T); it waits for each block's flag before it fetches that block.
//   sdep: block b of a pair update (TSMQR, TTMQR) reads and writes only rows
//   b ib .. b ib + ib - 1 of its C1 tile.  If the previous writer of that
//   tile slab is a pair update with the same pivot row (C1 in both) or the
//   UNMQR of the pivot row (whose block b finishes rows up to b ib + ib - 1
//   for good), block b only needs the previous writer's progress past its
//   own block b; writers publish their progress after every block.
// Streamed predecessors still count in the priorities and the level order.
//
// early (with pblk > 1): a panel block subtask releases its successors once
// it has factored its block and applied it to the next block's columns
// (the look-ahead), and updates the rest of its tiles after that.  Block b
// of a panel task then starts after the early release of block b - 1 and of
// block b of the earlier panel tasks on its triangles (their factored
// columns and look-ahead columns are final, and so is everything their own
// earlier blocks wrote); it waits for the completion of block b - 1 before
// its look-ahead (block b - 1 updated the next block's columns last) and
// for the completion of block b of the earlier panel tasks before the rest
// of its tiles (they updated the same rows of those columns last).  Every
// block waits at both points even when it has nothing to update, so the
// completion of block b still implies the completion of everything block b
// waited for.  Streamed update subtasks only read the reflectors and T of
// panel block b, which are final at its early release.
void make_exec_plan(const Plan& plan, int nslab, int order, const double w[6], ExecPlan& ex, int pblk, bool stream,
                    bool early, int workers) {
  const int p = plan.p, q = plan.q, S = nslab;
  ex = ExecPlan();
  ex.nslab = S;
  ex.pblk = pblk;
  const size_t ntile = static_cast<size_t>(p) * q;
  std::vector<int32_t> up(ntile * S, -1), lo(ntile * S, -1);
  auto slot = [&](int r, int c, int s) { return (static_cast<size_t>(r - 1) * q + (c - 1)) * S + s; };

  std::vector<SubTask> sub;  // emission order
  std::vector<std::vector<int32_t>> pre;
  std::vector<int32_t> task_of;
  std::vector<int32_t> sdep, pfirst;  // streamed C1 writer, panel block 0 (emission order), or -1
  sub.reserve(plan.tasks.size() * 2);
  stream = stream && pblk > 1;
  early = early && pblk > 1;

  std::vector<int32_t> first_blk;  // panel subtasks: id of block 0 of the task; -1 otherwise
  auto add = [&](const Task& t, int32_t tidx, int slab, std::vector<int32_t>&& d) {
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    if (!d.empty() && d.front() < 0) d.erase(d.begin(), std::upper_bound(d.begin(), d.end(), -1));
    // an entry that is also waited for in full at the start needs no other
    // entry for the same predecessor
    std::vector<int32_t> plain;
    for (int32_t x : d)
      if (dep_bits(x) == 0) plain.push_back(x);
    d.erase(std::remove_if(d.begin(), d.end(),
                           [&](int32_t x) {
                             return dep_bits(x) != 0 && std::binary_search(plain.begin(), plain.end(), dep_index(x));
                           }),
            d.end());
    sub.push_back({t.kind, t.i - 1, t.piv > 0 ? t.piv - 1 : 0, t.k - 1, t.j > 0 ? t.j - 1 : 0, slab, 0, 0, -1, -1});
    pre.push_back(std::move(d));
    task_of.push_back(tidx);
    first_blk.push_back(-1);
    sdep.push_back(-1);
    pfirst.push_back(-1);
    return static_cast<int32_t>(sub.size()) - 1;
  };
  // The last panel block subtask w among the reflector writers d (a panel
  // task split into pblk blocks): returns its block 0, and drops w from d.
  auto take_panel = [&](std::vector<int32_t>& d) -> int32_t {
    if (!stream) return -1;
    int32_t w = -1;
    for (int32_t x : d)
      if (x >= 0 && first_blk[x] >= 0) w = (w < 0 || x > w) ? x : w;
    if (w < 0) return -1;
    const int32_t f = first_blk[w];
    if (w != f + pblk - 1) return -1;
    d.erase(std::remove(d.begin(), d.end(), w), d.end());
    return f;
  };
  // A panel task: one subtask, or pblk block subtasks; returns the id of the
  // last.  d_full: writers the task waits for as a whole (from block 0);
  // d_blk: writers of the triangles of its pivot (and, for TTQRT, of its
  // killed tile), which block b waits for block by block when they are
  // block subtasks of an earlier panel task.
  auto add_panel = [&](const Task& t, int32_t tidx, std::vector<int32_t>&& d_full, std::vector<int32_t>&& d_blk) {
    if (pblk <= 1) {
      d_full.insert(d_full.end(), d_blk.begin(), d_blk.end());
      return add(t, tidx, -1, std::move(d_full));
    }
    std::vector<int32_t> other, panel_first;
    for (int32_t x : d_full)
      if (x >= 0) other.push_back(x);
    for (int32_t x : d_blk) {
      if (x < 0) continue;
      if (first_blk[x] >= 0)
        panel_first.push_back(first_blk[x]);
      else
        other.push_back(x);
    }
    std::sort(panel_first.begin(), panel_first.end());
    panel_first.erase(std::unique(panel_first.begin(), panel_first.end()), panel_first.end());
    int32_t first = -1, prev = -1;
    for (int b = 0; b < pblk; ++b) {
      std::vector<int32_t> db;
      if (b == 0) db = other;
      if (early) {
        if (prev >= 0) {
          db.push_back(prev | DEP_EARLY);
          db.push_back(prev | DEP_STAGE1);
        }
        for (int32_t f : panel_first) {
          db.push_back((f + b) | DEP_EARLY);
          db.push_back((f + b) | DEP_STAGE2);
        }
      } else {
        if (prev >= 0) db.push_back(prev);
        for (int32_t f : panel_first) db.push_back(f + b);
      }
      prev = add(t, tidx, b, std::move(db));
      if (b == 0) first = prev;
      first_blk[prev] = first;
    }
    return prev;
  };

  for (size_t ti = 0; ti < plan.tasks.size(); ++ti) {
    const Task& t = plan.tasks[ti];
    const int32_t tid = static_cast<int32_t>(ti);
    switch (t.kind) {
      case K_GEQRT: {
        std::vector<int32_t> d;
        for (int s = 0; s < S; ++s) {
          d.push_back(up[slot(t.i, t.k, s)]);
          d.push_back(lo[slot(t.i, t.k, s)]);
        }
        const int32_t id = add_panel(t, tid, std::move(d), {});
        for (int s = 0; s < S; ++s) up[slot(t.i, t.k, s)] = lo[slot(t.i, t.k, s)] = id;
        break;
      }
      case K_TTQRT:
      case K_TSQRT: {
        std::vector<int32_t> d_full, d_blk;
        for (int s = 0; s < S; ++s) {
          d_blk.push_back(up[slot(t.piv, t.k, s)]);
          if (t.kind == K_TTQRT) {
            d_blk.push_back(up[slot(t.i, t.k, s)]);
          } else {
            d_full.push_back(up[slot(t.i, t.k, s)]);
            d_full.push_back(lo[slot(t.i, t.k, s)]);
          }
        }
        const int32_t id = add_panel(t, tid, std::move(d_full), std::move(d_blk));
        for (int s = 0; s < S; ++s) {
          up[slot(t.piv, t.k, s)] = id;
          up[slot(t.i, t.k, s)] = id;
          if (t.kind == K_TSQRT) lo[slot(t.i, t.k, s)] = id;
        }
        break;
      }
      case K_UNMQR: {
        for (int s = 0; s < S; ++s) {
          std::vector<int32_t> dv, d;
          for (int s2 = 0; s2 < S; ++s2) dv.push_back(lo[slot(t.i, t.k, s2)]);
          const int32_t pf = take_panel(dv);
          d = dv;
          d.push_back(up[slot(t.i, t.j, s)]);
          d.push_back(lo[slot(t.i, t.j, s)]);
          const int32_t id = add(t, tid, s, std::move(d));
          pfirst[id] = pf;
          up[slot(t.i, t.j, s)] = lo[slot(t.i, t.j, s)] = id;
        }
        break;
      }
      default: {  // TSMQR / TTMQR
        for (int s = 0; s < S; ++s) {
          std::vector<int32_t> dv, d;
          for (int s2 = 0; s2 < S; ++s2) {
            dv.push_back(up[slot(t.i, t.k, s2)]);
            if (t.kind == K_TSMQR) dv.push_back(lo[slot(t.i, t.k, s2)]);
          }
          const int32_t pf = take_panel(dv);
          d = dv;
          const int32_t c2u = up[slot(t.i, t.j, s)], c2l = lo[slot(t.i, t.j, s)];
          int32_t c1 = up[slot(t.piv, t.j, s)];
          const bool c1_stream = stream && c1 >= 0 && c1 == lo[slot(t.piv, t.j, s)] && c1 != c2u && c1 != c2l &&
                                 std::find(d.begin(), d.end(), c1) == d.end() &&
                                 ((sub[c1].kind == K_UNMQR && sub[c1].i == t.piv - 1) ||
                                  ((sub[c1].kind == K_TSMQR || sub[c1].kind == K_TTMQR) && sub[c1].piv == t.piv - 1));
          if (!c1_stream) {
            d.push_back(c1);
            d.push_back(lo[slot(t.piv, t.j, s)]);
          }
          d.push_back(c2u);
          d.push_back(c2l);
          const int32_t id = add(t, tid, s, std::move(d));
          pfirst[id] = pf;
          if (c1_stream) sdep[id] = c1;
          up[slot(t.piv, t.j, s)] = lo[slot(t.piv, t.j, s)] = id;
          up[slot(t.i, t.j, s)] = lo[slot(t.i, t.j, s)] = id;
        }
        break;
      }
    }
  }

  // Priorities: ASAP start (order 0), ALAP start (order 1) or largest bottom
  // level first (order 2) of each subtask, with per-kind weights (updates
  // divided among their slabs, panel tasks among their blocks); or (order 3)
  // the start order of a list schedule of the subtasks on `workers`
  // workgroups that starts, whenever a workgroup is free, the ready subtask
  // of largest bottom level (sim_order).
  const size_t n = sub.size();
  std::vector<double> wt(n), est(n, 0.0), lst(n, 0.0);
  for (size_t s = 0; s < n; ++s) {
    const int kd = sub[s].kind;
    const bool is_upd = (kd == K_UNMQR || kd == K_TSMQR || kd == K_TTMQR);
    wt[s] = is_upd ? w[kd] / S : w[kd] / (sub[s].slab >= 0 ? pblk : 1);
  }
  // All predecessors, the streamed ones included, order the subtasks.
  std::vector<std::vector<int32_t>> allp(n);
  for (size_t s = 0; s < n; ++s) {
    for (int32_t d : pre[s]) allp[s].push_back(dep_index(d));
    if (sdep[s] >= 0) allp[s].push_back(sdep[s]);
    if (pfirst[s] >= 0)
      for (int b = 0; b < pblk; ++b) allp[s].push_back(pfirst[s] + b);
  }
  double span = 0.0;
  for (size_t s = 0; s < n; ++s) {
    double st = 0.0;
    for (int32_t d : allp[s]) st = std::max(st, est[d] + wt[d]);
    est[s] = st;
    span = std::max(span, st + wt[s]);
  }
  std::vector<std::vector<int32_t>> succ(n);
  for (size_t s = 0; s < n; ++s)
    for (int32_t d : allp[s]) succ[d].push_back(static_cast<int32_t>(s));
  for (size_t s = n; s-- > 0;) {
    double lf = span;
    for (int32_t c : succ[s]) lf = std::min(lf, lst[c]);
    lst[s] = lf - wt[s];
  }
  // Bottom level: longest path from the start of the subtask to the end.
  std::vector<double> bl(n, 0.0);
  for (size_t s = n; s-- > 0;) {
    double m = 0.0;
    for (int32_t c : succ[s]) m = std::max(m, bl[c]);
    bl[s] = m + wt[s];
  }
  std::vector<double> negbl(n);
  for (size_t s = 0; s < n; ++s) negbl[s] = -bl[s];
  std::vector<double> simk;
  if (order == 3 && workers > 0) simk = sim_order(sub, pre, sdep, pfirst, pblk, wt, bl, workers);
  const std::vector<double>& key = (order == 1) ? lst : (order == 2 ? negbl : (order == 3 && workers > 0 ? simk : est));
  std::vector<int32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
    if (key[a] != key[b]) return key[a] < key[b];
    return a < b;
  });
  std::vector<int32_t> pos(n);
  for (size_t r = 0; r < n; ++r) pos[perm[r]] = static_cast<int32_t>(r);

  ex.sub.resize(n);
  ex.deps.clear();
  ex.key.resize(n);
  ex.wt.resize(n);
  for (size_t r = 0; r < n; ++r) {
    ex.key[r] = key[perm[r]];
    ex.wt[r] = wt[perm[r]];
  }
  for (size_t r = 0; r < n; ++r) {
    const int32_t s = perm[r];
    SubTask st = sub[s];
    st.dep_begin = static_cast<int32_t>(ex.deps.size());
    for (int32_t d : pre[s]) ex.deps.push_back(pos[dep_index(d)] | dep_bits(d));
    st.dep_end = static_cast<int32_t>(ex.deps.size());
    st.sdep = sdep[s] >= 0 ? pos[sdep[s]] : -1;
    st.pdep = -1;
    if (pfirst[s] >= 0) {
      st.pdep = static_cast<int32_t>(ex.deps.size());
      for (int b = 0; b < pblk; ++b) ex.deps.push_back(pos[pfirst[s] + b] | (early ? DEP_EARLY : 0));
    }
    ex.sub[r] = st;
  }

  // Depth levels for the level-synchronous launch path (streamed
  // predecessors run in earlier levels).
  std::vector<int32_t> depth(n, 0);
  int32_t maxd = 0;
  for (size_t r = 0; r < n; ++r) {
    int32_t dd = 0;
    for (int32_t d : stream_preds(ex, r)) dd = std::max(dd, depth[d] + 1);
    depth[r] = dd;
    maxd = std::max(maxd, dd);
  }
  ex.level_ptr.assign(maxd + 2, 0);
  for (size_t r = 0; r < n; ++r) ex.level_ptr[depth[r] + 1]++;
  for (int32_t l = 0; l <= maxd; ++l) ex.level_ptr[l + 1] += ex.level_ptr[l];
  ex.level_order.assign(n, 0);
  std::vector<int32_t> fill(ex.level_ptr.begin(), ex.level_ptr.end() - 1);
  for (size_t r = 0; r < n; ++r) ex.level_order[fill[depth[r]]++] = static_cast<int32_t>(r);
}

}  // namespace tqr

namespace tqr {

void make_apply_plan(const Plan& plan, int trans, int nslab, ExecPlan& ex) {
  ex = ExecPlan();
  ex.nslab = nslab;
  std::vector<int32_t> order;
  for (size_t t = 0; t < plan.tasks.size(); ++t) {
    const int k = plan.tasks[t].kind;
    if (k == K_GEQRT || k == K_TSQRT || k == K_TTQRT) order.push_back(static_cast<int32_t>(t));
  }
  if (!trans) std::reverse(order.begin(), order.end());
  std::vector<int32_t> last(static_cast<size_t>(plan.p) * nslab, -1);
  for (int32_t t : order) {
    const Task& tk = plan.tasks[t];
    const int kind = tk.kind == K_GEQRT ? 6 : (tk.kind == K_TSQRT ? 7 : 8);
    for (int s = 0; s < nslab; ++s) {
      SubTask st{kind, tk.i - 1, tk.piv > 0 ? tk.piv - 1 : 0, tk.k - 1, 0, s, 0, 0, -1, -1};
      st.dep_begin = static_cast<int32_t>(ex.deps.size());
      const int32_t a = last[static_cast<size_t>(tk.i - 1) * nslab + s];
      const int32_t b = tk.piv > 0 ? last[static_cast<size_t>(tk.piv - 1) * nslab + s] : -1;
      if (a >= 0) ex.deps.push_back(a);
      if (b >= 0 && b != a) ex.deps.push_back(b);
      st.dep_end = static_cast<int32_t>(ex.deps.size());
      const int32_t id = static_cast<int32_t>(ex.sub.size());
      ex.sub.push_back(st);
      last[static_cast<size_t>(tk.i - 1) * nslab + s] = id;
      if (tk.piv > 0) last[static_cast<size_t>(tk.piv - 1) * nslab + s] = id;
    }
  }
  const size_t n = ex.sub.size();
  std::vector<int32_t> depth(n, 0);
  int32_t maxd = 0;
  for (size_t r = 0; r < n; ++r) {
    int32_t dd = 0;
    for (int32_t e = ex.sub[r].dep_begin; e < ex.sub[r].dep_end; ++e) dd = std::max(dd, depth[ex.deps[e]] + 1);
    depth[r] = dd;
    maxd = std::max(maxd, dd);
  }
  ex.level_ptr.assign(maxd + 2, 0);
  for (size_t r = 0; r < n; ++r) ex.level_ptr[depth[r] + 1]++;
  for (int32_t l = 0; l <= maxd; ++l) ex.level_ptr[l + 1] += ex.level_ptr[l];
  ex.level_order.assign(n, 0);
  std::vector<int32_t> fill(ex.level_ptr.begin(), ex.level_ptr.end() - 1);
  for (size_t r = 0; r < n; ++r) ex.level_order[fill[depth[r]]++] = static_cast<int32_t>(r);
}

void make_factor_apply_plan(const Plan& plan, const ExecPlan& fac, int nslab, int nslab_b, double w_apply,
                            ExecPlan& out) {
  ExecPlan ap;
  make_apply_plan(plan, 1, nslab_b, ap);
  const size_t nf = fac.sub.size(), na = ap.sub.size(), n = nf + na;
  // Panel subtask of each (kind, i, k).
  std::map<std::tuple<int, int, int>, int32_t> panel;
  for (size_t t = 0; t < nf; ++t) {
    const SubTask& s = fac.sub[t];
    // the subtask that completes the panel task (the whole task, or its last block)
    if ((s.kind == K_GEQRT || s.kind == K_TSQRT || s.kind == K_TTQRT) && (s.slab < 0 || s.slab == fac.pblk - 1))
      panel[{s.kind, s.i, s.k}] = static_cast<int32_t>(t);
  }
  std::vector<std::vector<int32_t>> pre(n);
  for (size_t t = 0; t < nf; ++t)
    for (int32_t e = fac.sub[t].dep_begin; e < fac.sub[t].dep_end; ++e) pre[t].push_back(fac.deps[e]);
  for (size_t a = 0; a < na; ++a) {
    const SubTask& s = ap.sub[a];
    for (int32_t e = s.dep_begin; e < s.dep_end; ++e) pre[nf + a].push_back(static_cast<int32_t>(nf) + ap.deps[e]);
    const int fk = s.kind == 6 ? K_GEQRT : (s.kind == 7 ? K_TSQRT : K_TTQRT);
    auto it = panel.find({fk, s.i, s.k});
    if (it != panel.end()) pre[nf + a].push_back(it->second);
  }
  // Dispatch order: the factorization subtasks keep theirs; an application
  // subtask goes right behind the last of its predecessors (its panel
  // subtask, the previous application on its rows), so the Q^T B chain
  // advances with the factorization instead of trailing it.
  std::vector<double> key(n);
  for (size_t t = 0; t < nf; ++t) key[t] = static_cast<double>(t);
  const double eps = 1.0 / static_cast<double>(na + 2);
  for (size_t a = 0; a < na; ++a) {
    double k = -1.0;
    for (int32_t d : pre[nf + a]) k = std::max(k, key[d]);
    key[nf + a] = k + eps;
  }
  std::vector<double> wt(n);
  for (size_t t = 0; t < nf; ++t) wt[t] = fac.wt[t];
  for (size_t a = 0; a < na; ++a) wt[nf + a] = w_apply;
  std::vector<int32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
    if (key[a] != key[b]) return key[a] < key[b];
    return a < b;
  });
  std::vector<int32_t> pos(n);
  for (size_t r = 0; r < n; ++r) pos[perm[r]] = static_cast<int32_t>(r);
  out = ExecPlan();
  out.nslab = nslab;
  out.pblk = fac.pblk;
  out.sub.resize(n);
  out.key.resize(n);
  out.wt.resize(n);
  for (size_t r = 0; r < n; ++r) {
    const int32_t t = perm[r];
    SubTask st = t < static_cast<int32_t>(nf) ? fac.sub[t] : ap.sub[t - nf];
    st.dep_begin = static_cast<int32_t>(out.deps.size());
    for (int32_t d : pre[t]) out.deps.push_back(pos[dep_index(d)] | dep_bits(d));
    st.dep_end = static_cast<int32_t>(out.deps.size());
    if (st.sdep >= 0) st.sdep = pos[st.sdep];
    if (st.pdep >= 0) {
      const int32_t old = st.pdep;
      st.pdep = static_cast<int32_t>(out.deps.size());
      for (int b = 0; b < fac.pblk; ++b) {
        const int32_t d = fac.deps[old + b];
        out.deps.push_back(pos[dep_index(d)] | dep_bits(d));
      }
    }
    out.sub[r] = st;
    out.key[r] = key[t];
    out.wt[r] = wt[t];
  }
  std::vector<int32_t> depth(n, 0);
  int32_t maxd = 0;
  for (size_t r = 0; r < n; ++r) {
    int32_t dd = 0;
    for (int32_t d : stream_preds(out, r)) dd = std::max(dd, depth[d] + 1);
    depth[r] = dd;
    maxd = std::max(maxd, dd);
  }
  out.level_ptr.assign(maxd + 2, 0);
  for (size_t r = 0; r < n; ++r) out.level_ptr[depth[r] + 1]++;
  for (int32_t l = 0; l <= maxd; ++l) out.level_ptr[l + 1] += out.level_ptr[l];
  out.level_order.assign(n, 0);
  std::vector<int32_t> fill(out.level_ptr.begin(), out.level_ptr.end() - 1);
  for (size_t r = 0; r < n; ++r) out.level_order[fill[depth[r]]++] = static_cast<int32_t>(r);
}

}  // namespace tqr
