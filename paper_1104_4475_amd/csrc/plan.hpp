// Host planner: elimination lists, kernel-task DAG, schedules and the
// executor's slab-level task table.
#pragma once

#include <cstdint>
#include <vector>

#include "depcode.hpp"

namespace tqr {

enum Kind : int32_t { K_GEQRT = 0, K_UNMQR = 1, K_TSQRT = 2, K_TSMQR = 3, K_TTQRT = 4, K_TTMQR = 5 };
enum Tree : int32_t {
  T_FLAT = 0, T_SAMEH_KUCK = 1, T_BINARY = 2, T_FIBONACCI = 3, T_GREEDY = 4, T_PLASMA = 5, T_ASAP = 6, T_GRASAP = 7,
  T_HADRI = 8
};
enum Family : int32_t { F_DEFAULT = 0, F_TT = 1, F_TS = 2 };

// Table 1 weights in units of nb^3/3 flops.
constexpr int kWeight[6] = {4, 6, 6, 12, 2, 6};

struct Elim { int32_t i, piv, k; };          // 1-based (Sec. 2.2)
struct Task { int32_t kind, i, piv, k, j; };  // 1-based, 0 in unused fields

struct Plan {
  int32_t p = 0, q = 0, tree = 0, bs = 1, family = F_TT;
  std::vector<Elim> elims;
  std::vector<Task> tasks;
  std::vector<int64_t> pred_ptr;   // CSR predecessors, ntasks + 1
  std::vector<int32_t> pred_idx;
  std::vector<int64_t> start, finish;
  int64_t cp = 0;
};

// Returns false on invalid (p, q, tree, bs).
bool valid_shape(int p, int q, int tree, int bs);
int resolve_family(int tree, int family);
bool make_elims(int p, int q, int tree, int bs, std::vector<Elim>& out);
bool make_plan(int p, int q, int tree, int bs, int family, Plan& plan);

// Executor task table.  Update tasks are split into column slabs of the
// C tiles; panel tasks stay whole.  Subtasks are stored in dispatch order
// (a topological order), dependencies index earlier subtasks.
struct SubTask {
  int32_t kind, i, piv, k, j;   // 0-based tile indices (i, piv, k, j)
  int32_t slab;                 // column slab of the C tiles (updates); for panel
                                // tasks the inner block it factors, -1 = all
  int32_t dep_begin, dep_end;   // range in deps[] of the predecessors waited for
                                // before the subtask starts
  int32_t sdep;                 // streamed predecessor (see make_exec_plan), or -1
  int32_t pdep;                 // offset in deps[] of the nb/ib panel block
                                // subtasks whose reflectors it streams, or -1
};

struct ExecPlan {
  std::vector<SubTask> sub;
  std::vector<int32_t> deps;
  std::vector<int32_t> level_ptr;    // subtasks grouped by DAG depth
  std::vector<int32_t> level_order;  // indices into sub, level by level
  std::vector<double> key;           // priority key of each subtask (ascending = earlier)
  std::vector<double> wt;            // weight of each subtask in the priorities
  int32_t nslab = 1;
  int32_t pblk = 1;                  // subtasks per panel task (inner blocks)
};

// order: 0 = ascending ASAP start time, 1 = ascending ALAP start time,
// 2 = descending bottom level (longest remaining path), 3 = start order of a
// list schedule on `workers` workgroups by descending bottom level among
// the ready subtasks (plan.cpp; needs workers > 0, else as 0).
// w: per-kind weights used for the priority (any positive values).
// pblk > 1 splits every panel task (GEQRT, TSQRT, TTQRT) into its pblk inner
// blocks of columns, one subtask each (see plan.cpp).
// stream (with pblk > 1): update subtasks follow their reflectors block by
// block (pdep) and pair updates follow the previous writer of their C1 tile
// block by block (sdep) instead of waiting for them to finish (plan.cpp).
// early (with pblk > 1): panel block subtasks release their successors
// after their look-ahead update and wait for the rest of their
// predecessors inside (plan.cpp); predecessor entries then carry the fields
// of depcode.hpp.
void make_exec_plan(const Plan& plan, int nslab, int order, const double w[6], ExecPlan& ex, int pblk = 1,
                    bool stream = false, bool early = false, int workers = 0);

// One executor plan for the factorization and Q^T B together: the
// subtasks of fac (built by make_exec_plan with the same nslab; their
// priority weights are fac.wt) and those of the Q^T application plan
// (make_apply_plan, trans = 1, nslab_b slabs of B), each application
// subtask also depending on the panel subtask that produces its
// reflectors.  Ordered by largest bottom level in the joint graph
// (application subtasks weigh w_apply).
void make_factor_apply_plan(const Plan& plan, const ExecPlan& fac, int nslab, int nslab_b, double w_apply,
                            ExecPlan& out);

// Application of Q^T (trans = 1) or Q (trans = 0) to p row tiles of a
// right-hand side with nslab column slabs: the reflector set of every panel
// task, in task order for Q^T and in reverse for Q, with dependencies on the
// row tiles it touches.  Kinds are 6 (GEQRT set), 7 (TS set), 8 (TT set).
void make_apply_plan(const Plan& plan, int trans, int nslab, ExecPlan& ex);

}  // namespace tqr
