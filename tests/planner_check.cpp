// Host check of the executor plans (built with the address and undefined
// behaviour sanitizers by tests/test_planner_exec.py): for a grid of shapes,
// trees, kernel families, slab counts, panel splits, streaming, early
// release and dispatch orders, every plan must be a valid executor input:
//   * every predecessor entry names an earlier subtask, with stage 0, 1 or 2;
//   * entries waited for inside a subtask (stages 1, 2) only occur on panel
//     block subtasks and pair with an early (or plain) start entry for the
//     same predecessor;
//   * streamed predecessors (sdep, pdep blocks) are earlier subtasks;
//   * the subtasks are the same for every dispatch order, with the same
//     predecessors (as sets of subtask identities);
//   * the joint factorization + Q^T B plan keeps all of this.
// Prints "ok <plans checked>" or the first failure, and exits nonzero then.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "plan.hpp"

using namespace tqr;

namespace {

using Key = std::tuple<int, int, int, int, int, int>;

Key key_of(const SubTask& s) { return Key{s.kind, s.i, s.piv, s.k, s.j, s.slab}; }

bool fail(const char* what, const std::string& where) {
  std::printf("FAIL %s (%s)\n", what, where.c_str());
  return false;
}

// Validity of one plan; fills edges with (successor, predecessor, bits).
bool check_plan(const ExecPlan& ex, const std::string& where, std::set<std::tuple<Key, Key, int>>* edges) {
  const int32_t n = static_cast<int32_t>(ex.sub.size());
  if (static_cast<int32_t>(ex.key.size()) != n || static_cast<int32_t>(ex.wt.size()) != n)
    return fail("key/weight size", where);
  std::set<Key> seen;
  for (int32_t t = 0; t < n; ++t) {
    const SubTask& s = ex.sub[t];
    if (!seen.insert(key_of(s)).second) return fail("duplicate subtask", where);
    if (s.dep_begin < 0 || s.dep_end < s.dep_begin || s.dep_end > static_cast<int32_t>(ex.deps.size()))
      return fail("dep range", where);
    const bool panel_blk = (s.kind == K_GEQRT || s.kind == K_TSQRT || s.kind == K_TTQRT) && s.slab >= 0;
    std::set<int32_t> start_idx;
    for (int32_t e = s.dep_begin; e < s.dep_end; ++e) {
      const int32_t d = ex.deps[e];
      if (d < 0 || dep_index(d) >= t) return fail("predecessor not earlier", where);
      if (dep_stage(d) == 3) return fail("stage 3", where);
      if (dep_stage(d) != 0 && !panel_blk) return fail("inside wait on a non-panel subtask", where);
      if (dep_stage(d) != 0 && dep_early(d)) return fail("early bit on an inside wait", where);
      if (dep_stage(d) == 0) start_idx.insert(dep_index(d));
      if (edges) edges->insert({key_of(s), key_of(ex.sub[dep_index(d)]), dep_bits(d)});
    }
    for (int32_t e = s.dep_begin; e < s.dep_end; ++e) {
      const int32_t d = ex.deps[e];
      if (dep_stage(d) != 0 && !start_idx.count(dep_index(d))) return fail("inside wait without a start entry", where);
    }
    if (s.sdep >= t) return fail("sdep not earlier", where);
    if (s.sdep >= 0 && edges) edges->insert({key_of(s), key_of(ex.sub[s.sdep]), -1});
    if (s.pdep >= 0) {
      if (s.pdep + ex.pblk > static_cast<int32_t>(ex.deps.size())) return fail("pdep range", where);
      for (int b = 0; b < ex.pblk; ++b) {
        const int32_t d = ex.deps[s.pdep + b];
        if (d < 0 || dep_index(d) >= t || dep_stage(d) != 0) return fail("pdep entry", where);
        const SubTask& pb = ex.sub[dep_index(d)];
        if (pb.slab != b) return fail("pdep block order", where);
        if (edges) edges->insert({key_of(s), key_of(pb), -2 - (dep_bits(d) != 0)});
      }
    }
  }
  return true;
}

}  // namespace

int main() {
  const double w[6] = {600, 144, 560, 212, 466, 156};
  const int shapes[][2] = {{1, 1}, {3, 1}, {6, 3}, {9, 9}, {12, 5}};
  const int trees[] = {T_FLAT, T_SAMEH_KUCK, T_BINARY, T_FIBONACCI, T_GREEDY, T_PLASMA, T_ASAP, T_GRASAP, T_HADRI};
  long checked = 0;
  for (const auto& sh : shapes) {
    const int p = sh[0], q = sh[1];
    for (int tree : trees) {
      for (int bs : {1, 3}) {
        if (!valid_shape(p, q, tree, bs)) continue;
        for (int fam : {F_TT, F_TS}) {
          Plan plan;
          if (!make_plan(p, q, tree, bs, fam, plan)) continue;
          for (int nslab : {1, 2}) {
            for (int pblk : {1, 8}) {
              for (int mode = 0; mode < 4; ++mode) {
                const bool stream = mode & 1, early = mode & 2;
                std::set<std::tuple<Key, Key, int>> ref;
                bool have_ref = false;
                for (int order = 0; order < 4; ++order) {
                  for (int workers : {1, 256}) {
                    if (order != 3 && workers != 1) continue;
                    char buf[160];
                    std::snprintf(buf, sizeof buf, "p %d q %d tree %d bs %d fam %d nslab %d pblk %d stream %d early %d order %d workers %d",
                                  p, q, tree, bs, fam, nslab, pblk, stream, early, order, workers);
                    ExecPlan ex;
                    make_exec_plan(plan, nslab, order, w, ex, pblk, stream, early, workers);
                    std::set<std::tuple<Key, Key, int>> edges;
                    if (!check_plan(ex, buf, &edges)) return 1;
                    if (!have_ref) {
                      ref = edges;
                      have_ref = true;
                    } else if (edges != ref) {
                      std::printf("FAIL edges depend on the dispatch order (%s)\n", buf);
                      return 1;
                    }
                    ExecPlan joint;
                    make_factor_apply_plan(plan, ex, nslab, 1, 10.0, joint);
                    if (!check_plan(joint, std::string(buf) + " joint", nullptr)) return 1;
                    if (joint.sub.size() <= ex.sub.size()) return fail("joint plan size", buf), 1;
                    checked += 2;
                  }
                }
              }
            }
          }
        }
      }
    }
  }
  std::printf("ok %ld\n", checked);
  return 0;
}
