// Host tables of the forward and backward sweeps (Sec. 5.2.2) for a plan:
// update-vector offsets, per-position gather lists of the fronts, offsets of
// the two packed layouts of F, the 64-row tasks of every level and the tile
// shape each level starts from.  Everything the sweeps' memory traffic depends
// on besides the plan itself and the sweep kernels is decided here.
#include "sweep_plan.hpp"

#include <algorithm>

namespace riga {

void build_sweep_plan(const Plan& P, const std::vector<int>& node_inst, SweepPlan& S) {
  const size_t nn = P.nf.size();
  S.voff.assign(nn + 1, 0);
  for (size_t v = 0; v < nn; ++v) S.voff[v + 1] = S.voff[v] + P.nb[v];
  // per front position, the children's update rows that land on it, in child order
  const size_t npos = (size_t)P.foff.back();
  std::vector<int> gcnt(npos + 1, 0);
  S.gptr.assign(npos + 1, 0);
  S.gidx.assign((size_t)S.voff.back(), 0);
  for (size_t v = 0; v < nn; ++v)
    for (int ci = P.coff[v]; ci < P.coff[v + 1]; ++ci) {
      const int c = P.clist[ci];
      for (int k = 0; k < P.nb[c]; ++k) ++gcnt[P.foff[v] + P.maps[P.moff[c] + k]];
    }
  for (size_t q = 0; q < npos; ++q) S.gptr[q + 1] = S.gptr[q] + gcnt[q];
  std::vector<int> fill(S.gptr.begin(), S.gptr.end() - 1);
  for (size_t v = 0; v < nn; ++v)
    for (int ci = P.coff[v]; ci < P.coff[v + 1]; ++ci) {
      const int c = P.clist[ci];
      for (int k = 0; k < P.nb[c]; ++k) S.gidx[fill[P.foff[v] + P.maps[P.moff[c] + k]]++] = S.voff[c] + k;
    }
  S.gsrc.assign(npos, int4{-1, 0, 0, 0});
  for (size_t v = 0; v < nn; ++v)
    for (int p = 0; p < P.nf[v]; ++p) {
      const size_t q = (size_t)P.foff[v] + p;
      const int cnt = S.gptr[q + 1] - S.gptr[q];
      S.gsrc[q] = int4{p < P.no[v] ? P.fdofs[q] : -1, cnt, cnt > 0 ? S.gidx[S.gptr[q]] : 0,
                       cnt == 2 ? S.gidx[S.gptr[q] + 1] : S.gptr[q]};
    }
  // sweep layouts, room for FP64 (groups of 2) and FP32 (groups of 4) entries:
  // the forward one without the zero triangle; the backward one too on levels
  // with at least SWEEP_TRI_TASKS backward tasks (bandwidth-bound), else the
  // full rectangle (measured faster where a level is latency-bound)
  S.ttri.assign(nn, 0);
  for (int lv = 0; lv < P.height; ++lv) {
    int64_t bt = 0;
    for (int k = P.level_off[lv]; k < P.level_off[lv + 1]; ++k) bt += (P.no[P.level_nodes[k]] + 63) / 64;
    if (bt >= SWEEP_TRI_TASKS)
      for (int k = P.level_off[lv]; k < P.level_off[lv + 1]; ++k) S.ttri[P.level_nodes[k]] = 1;
  }
  S.lpoff.assign(nn + 1, 0);
  S.tpoff.assign(nn + 1, 0);
  for (size_t v = 0; v < nn; ++v) {
    const int nf = P.nf[v], no = P.no[v];
    // node starts on 16-element (128-byte FP64) boundaries
    auto up16 = [](int64_t e) { return (e + 15) / 16 * 16; };
    S.lpoff[v + 1] = S.lpoff[v] + up16(std::max(lp_size(nf, no, 2), lp_size(nf, no, 4)));
    S.tpoff[v + 1] = S.tpoff[v] + up16(S.ttri[v] ? std::max(tp_size(nf, no, 2), tp_size(nf, no, 4))
                                                 : (int64_t)((nf + 3) / 4 * 4) * no);
  }
  // slack past the last node: a forward task of a node without own dofs
  // reads (and discards) one round at the node's offset
  const int64_t slack = ((int64_t)P.max_front + 64) * 4;
  S.lpsize = S.lpoff.back() + slack;
  S.tpsize = S.tpoff.back() + slack;
  // Row tasks: blocks of 64 consecutive rows of one node.  Within a level the
  // tasks are launched largest first (columns a forward task reads: up to its
  // last row's diagonal; rows a backward task reads: from its first column
  // down), so the short ones fill the tail.
  S.ftasks.clear();
  S.btasks.clear();
  S.ftask_off.assign(P.height + 1, 0);
  S.btask_off.assign(P.height + 1, 0);
  S.fvar.assign(P.height, 0);
  S.bvar.assign(P.height, 0);
  auto task = [&](int v, int r0, int r1, int64_t poff) {
    SweepTask k{};
    k.v = v; k.r0 = r0; k.r1 = r1; k.nf = P.nf[v]; k.no = P.no[v]; k.foff = P.foff[v];
    k.voff = S.voff[v]; k.inst = node_inst.empty() ? 0 : node_inst[v]; k.poff = poff;
    return k;
  };
  for (int lv = 0; lv < P.height; ++lv) {
    const size_t f0 = S.ftasks.size(), b0 = S.btasks.size();
    for (int k = P.level_off[lv]; k < P.level_off[lv + 1]; ++k) {
      const int v = P.level_nodes[k];
      for (int r = 0; r < P.nf[v]; r += 64) S.ftasks.push_back(task(v, r, std::min(r + 64, P.nf[v]), S.lpoff[v]));
      for (int r = 0; r < P.no[v]; r += 64) S.btasks.push_back(task(v, r, std::min(r + 64, P.no[v]), S.tpoff[v]));
    }
    std::stable_sort(S.ftasks.begin() + f0, S.ftasks.end(), [](const SweepTask& x, const SweepTask& y) {
      return std::min(x.r1, x.no) > std::min(y.r1, y.no);
    });
    std::stable_sort(S.btasks.begin() + b0, S.btasks.end(), [](const SweepTask& x, const SweepTask& y) {
      return x.nf - x.r0 > y.nf - y.r0;
    });
    S.ftask_off[lv + 1] = (int)S.ftasks.size();
    S.btask_off[lv + 1] = (int)S.btasks.size();
    S.fvar[lv] = sweep_default_variant(S.ftask_off[lv + 1] - S.ftask_off[lv], true);
    S.bvar[lv] = sweep_default_variant(S.btask_off[lv + 1] - S.btask_off[lv], false);
  }
}

}  // namespace riga
