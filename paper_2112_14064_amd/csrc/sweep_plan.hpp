// Host tables of the solve sweeps (see sweep_plan.cpp).
#pragma once
#include <cstdint>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

namespace riga {

struct SweepPlan {
  std::vector<int> voff;                 // per node: first row of its update vector (nn + 1)
  std::vector<int> gptr, gidx;           // per front position: update rows added to it
  std::vector<int4> gsrc;                // per front position: {dof or -1, count, first row,
                                         //  second row (count 2) or gptr (count > 2)}
  std::vector<int64_t> lpoff, tpoff;     // per node: packed forward / backward layouts of F (nn + 1)
  std::vector<unsigned char> ttri;       // per node: backward layout without the zero triangle
  int64_t lpsize = 0, tpsize = 0;        // entries of the layouts, with slack
  std::vector<SweepTask> ftasks, btasks; // 64-row tasks grouped by level
  std::vector<int> ftask_off, btask_off; // level lv: tasks [off[lv], off[lv + 1])
  std::vector<int> fvar, bvar;           // tile shape per level (sweep_variant)
};

// node_inst: problem of every node of a forest, or empty.
void build_sweep_plan(const Plan& P, const std::vector<int>& node_inst, SweepPlan& S);

}  // namespace riga
