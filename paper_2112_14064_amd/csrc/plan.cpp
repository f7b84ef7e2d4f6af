// Host-side symbolic plan (integer work only; no device calls).
//
// The nested-dissection tree follows the observation of Sec. 3.3: in rIGA the
// C^0 hyperplanes coincide with the separators of a multifrontal solver, so
// the domain is bisected along hyperplanes until single macroelements remain;
// macroelements longer than the leaf size are bisected further at element
// interfaces.
// A separator holds every function whose support crosses the cutting line:
// one function thick at a C^0 hyperplane, p functions thick at an ordinary
// element interface of maximum-continuity IGA.
#include "plan.hpp"

#include <algorithm>
#include <functional>

namespace riga {

void Space1D::build(int p_, int ne_, int s_, int mult_, bool dirichlet) {
  build_ends(p_, ne_, s_, mult_, dirichlet, dirichlet);
}

void Space1D::build_ends(int p_, int ne_, int s_, int mult_, bool drop_first, bool drop_last) {
  p = p_; ne = ne_; s = s_;
  mult = mult_ < 0 ? p : mult_;
  off = drop_first ? 1 : 0;
  knots.clear();
  for (int i = 0; i <= p; ++i) knots.push_back(0);
  for (int k = 1; k < ne; ++k) {
    int m = (s > 0 && k % s == 0) ? mult : 1;
    for (int r = 0; r < m; ++r) knots.push_back(k);
  }
  for (int i = 0; i <= p; ++i) knots.push_back(ne);
  nall = (int)knots.size() - p - 1;
  n = nall - off - (drop_last ? 1 : 0);
  sup0.resize(n); sup1.resize(n);
  for (int d = 0; d < n; ++d) {
    sup0[d] = knots[d + off];
    sup1[d] = knots[d + off + p + 1];
  }
  lo.resize(n); hi.resize(n);
  for (int d = 0; d < n; ++d) {
    int a = d, b = d;
    while (a > 0 && std::max(sup0[a - 1], sup0[d]) < std::min(sup1[a - 1], sup1[d])) --a;
    while (b + 1 < n && std::max(sup0[b + 1], sup0[d]) < std::min(sup1[b + 1], sup1[d])) ++b;
    lo[d] = a; hi[d] = b;
  }
  first.resize(ne);
  for (int e = 0; e < ne; ++e) {
    int cnt = (int)(std::upper_bound(knots.begin(), knots.end(), e) - knots.begin());
    first[e] = cnt - 1 - p;   // span index minus p
  }
}

namespace {

// Cut position strictly inside (lo, hi).  rIGA boxes are cut at the C^0
// hyperplane nearest the middle; a box without an interior hyperplane (inside
// one macroelement) and every IGA box is cut at its middle element interface
// while it is longer than `leaf` elements (the separator there is p functions
// thick, as in maximum-continuity IGA).
int pick_cut(int lo, int hi, int s, int leaf) {
  int mid2 = lo + hi;  // twice the midpoint
  int best = -1, bestd = 1 << 30;
  if (s > 0) {
    for (int c = (lo / s + 1) * s; c < hi; c += s) {
      int d = std::abs(2 * c - mid2);
      if (d < bestd) { bestd = d; best = c; }
    }
    if (best >= 0) return best;
  }
  if (hi - lo > leaf) best = (lo + hi) / 2;
  return best;
}

}  // namespace

void Plan::symbolic(std::vector<int64_t>* colcount, int64_t& nnz_l, double& flops) const {
  const int64_t nd = ndof;
  const int n = sp.n;
  std::vector<int64_t> dof_at(nd);
  for (int64_t d = 0; d < nd; ++d) dof_at[elim_pos[d]] = d;
  // elimination tree by path compression (Liu): for row i, every earlier
  // column k coupled to i reaches i through its root
  std::vector<int64_t> parent(nd, -1), anc(nd, -1), cnt(nd, 1), mark(nd, -1);
  auto neighbours = [&](int64_t i, auto&& f) {
    const int64_t d = dof_at[i];
    if (!col.empty()) {
      for (int64_t q = rowptr[d]; q < rowptr[d + 1]; ++q) {
        const int64_t k = elim_pos[col[q]];
        if (k < i) f(k);
      }
      return;
    }
    const int x = (int)(d % n), y = (int)(d / n);
    for (int jj = sp.lo[y]; jj <= sp.hi[y]; ++jj)
      for (int ii = sp.lo[x]; ii <= sp.hi[x]; ++ii) {
        const int64_t k = elim_pos[(int64_t)jj * n + ii];
        if (k < i) f(k);
      }
  };
  for (int64_t i = 0; i < nd; ++i) {
    neighbours(i, [&](int64_t k) {
      int64_t r = k;
      while (anc[r] != -1 && anc[r] != i) {
        const int64_t t = anc[r];
        anc[r] = i;
        r = t;
      }
      if (anc[r] == -1) {
        anc[r] = i;
        parent[r] = i;
      }
    });
  }
  // row i of L is the union of the etree paths from its coupled columns up to
  // i (the row subtree): every column met on them gains the entry (i, j)
  for (int64_t i = 0; i < nd; ++i) {
    mark[i] = i;
    neighbours(i, [&](int64_t k) {
      for (int64_t j = k; mark[j] != i; j = parent[j]) {
        mark[j] = i;
        ++cnt[j];
      }
    });
  }
  nnz_l = 0;
  flops = 0.0;
  for (int64_t j = 0; j < nd; ++j) {
    nnz_l += cnt[j];
    const double c = (double)(cnt[j] - 1);
    flops += c * c + 2.0 * c;
  }
  if (colcount) *colcount = std::move(cnt);
}

void Plan::ensure_symbolic() {
  if (sym_nnz_l >= 0) return;
  symbolic(nullptr, sym_nnz_l, sym_flops);
}

void Plan::amalgamate() {
  const int nn = (int)nodes.size();
  if (amalg_group < 2 || nn < 2) return;
  const int root = nn - 1;
  // depth from the root and the number of nodes at every depth
  std::vector<int> depth(nn, 0), count;
  for (int v = root; v >= 0; --v) {
    for (int c : nodes[v].children) depth[c] = depth[v] + 1;
  }
  for (int v = 0; v < nn; ++v) {
    if ((int)count.size() <= depth[v]) count.resize(depth[v] + 1, 0);
    ++count[depth[v]];
  }
  // the top depths with at most amalg_max nodes are grouped by amalg_group
  int dtop = 0;
  while (dtop < (int)count.size() && count[dtop] <= amalg_max) ++dtop;
  // group heads: depths that are multiples of amalg_group; a head takes its
  // group only while the group's own dofs stay within amalg_own (large fronts
  // near the root of big meshes are bandwidth-bound: merging them only adds
  // work)
  std::vector<int> rep(nn), gown(nn, 0);
  for (int v = 0; v < nn; ++v) {            // postorder: descendants first
    const int d = depth[v];
    gown[v] = (int)nodes[v].own.size();
    if (d < dtop && d % amalg_group != 0) continue;
    // own dofs of the descendants within the group
    std::function<int(int)> sum = [&](int u) {
      int t = 0;
      for (int c : nodes[u].children)
        if (depth[c] < dtop && depth[c] % amalg_group != 0) t += (int)nodes[c].own.size() + sum(c);
      return t;
    };
    gown[v] += sum(v);
  }
  for (int v = root; v >= 0; --v) {
    const int d = depth[v];
    if (d < dtop && d % amalg_group != 0 && rep[nodes[v].parent] == nodes[v].parent &&
        gown[nodes[v].parent] <= amalg_own)
      rep[v] = nodes[v].parent;
    else if (d < dtop && d % amalg_group != 0 && rep[nodes[v].parent] != nodes[v].parent)
      rep[v] = rep[nodes[v].parent];
    else
      rep[v] = v;
  }
  bool any = false;
  for (int v = 0; v < nn; ++v) any |= rep[v] != v;
  if (!any) return;
  // the merged tree: own dofs of a group in postorder (children first),
  // children = the members' children outside the group
  std::vector<std::vector<int>> kids(nn), owns(nn);
  for (int v = 0; v < nn; ++v) {           // postorder: members before their group head
    const int g = rep[v];
    owns[g].insert(owns[g].end(), nodes[v].own.begin(), nodes[v].own.end());
    for (int c : nodes[v].children)
      if (rep[c] == c) kids[g].push_back(c);
  }
  std::vector<int> order;
  std::function<void(int)> dfs = [&](int v) {
    for (int c : kids[v]) dfs(c);
    order.push_back(v);
  };
  dfs(root);
  std::vector<int> newid(nn, -1);
  for (size_t k = 0; k < order.size(); ++k) newid[order[k]] = (int)k;
  std::vector<Node> out(order.size());
  for (size_t k = 0; k < order.size(); ++k) {
    const int v = order[k];
    Node nd = nodes[v];
    nd.own = std::move(owns[v]);
    std::sort(nd.own.begin(), nd.own.end());
    nd.children.clear();
    for (int c : kids[v]) nd.children.push_back(newid[c]);
    nd.parent = -1;
    nd.post = (int)k;
    out[k] = std::move(nd);
  }
  for (auto& nd : out)
    for (int c : nd.children) out[c].parent = nd.post;
  for (auto& nd : out) {
    nd.first_desc = nd.post;
    nd.height = 0;
    for (int c : nd.children) {
      nd.first_desc = std::min(nd.first_desc, out[c].first_desc);
      nd.height = std::max(nd.height, out[c].height + 1);
    }
  }
  nodes = std::move(out);
  height = nodes.back().height + 1;
  for (int64_t d = 0; d < ndof; ++d) node_of_dof[d] = newid[rep[node_of_dof[d]]];
}

int Plan::build(int p, int ne, int s, int leaf) {
  if (p < 1 || p > 8 || ne < 2) return -1;
  if (s < 0 || (s > 0 && ne % s != 0)) return -1;
  if (leaf <= 0) leaf = 8;
  leaf_size = leaf;
  sp.build(p, ne, s);
  n1d = sp.n;
  if (n1d < 1) return -1;
  ndof = n1d * n1d;
  const int n = sp.n;

  rowptr.assign(ndof + 1, 0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      int64_t r = (int64_t)j * n + i;
      rowptr[r + 1] = rowptr[r] + (int64_t)(sp.hi[i] - sp.lo[i] + 1) * (sp.hi[j] - sp.lo[j] + 1);
    }
  nnz = rowptr[ndof];

  return finish(ne, s, leaf,
                [&](int64_t d, int& x0, int& x1, int& y0, int& y1) {
                  const int i = (int)(d % n), j = (int)(d / n);
                  x0 = sp.sup0[i]; x1 = sp.sup1[i]; y0 = sp.sup0[j]; y1 = sp.sup1[j];
                },
                [&](int64_t d, auto&& f) {
                  const int i = (int)(d % n), j = (int)(d / n);
                  for (int jj = sp.lo[j]; jj <= sp.hi[j]; ++jj)
                    for (int ii = sp.lo[i]; ii <= sp.hi[i]; ++ii) f((int64_t)jj * n + ii);
                });
}

int Plan::build_hcurl(int p, int ne, int s, int leaf, bool pec) {
  if (p < 2 || p > 8 || ne < 2) return -1;
  if (s < 0 || (s > 0 && ne % s != 0)) return -1;
  kind = pec ? SPACE_HCURL : SPACE_HCURL_FREE;
  // component 0: S^{p-1} (x) S^p (eq. HcurlBasis), component 1: S^p (x) S^{p-1};
  // both degrees carry the hyperplane knots with multiplicity p - 1
  cx[0].build(p - 1, ne, s, p - 1, false);
  cy[0].build(p, ne, s, p - 1, pec);
  cx[1].build(p, ne, s, p - 1, pec);
  cy[1].build(p - 1, ne, s, p - 1, false);
  return build_vector(ne, s, leaf);
}

int Plan::build_hdiv(int p, int ne, int s, int leaf, int absorbing) {
  if (p < 2 || p > 8 || ne < 2 || absorbing < 0 || absorbing > 15) return -1;
  if (s < 0 || (s > 0 && ne % s != 0)) return -1;
  kind = SPACE_HDIV;
  walls = absorbing;
  // component 0: S^p (x) S^{p-1} (eq. HdivBasis), component 1: S^{p-1} (x) S^p;
  // the normal direction's end functions go with the rigid walls
  cx[0].build_ends(p, ne, s, p - 1, !(absorbing & WALL_LEFT), !(absorbing & WALL_RIGHT));
  cy[0].build(p - 1, ne, s, p - 1, false);
  cx[1].build(p - 1, ne, s, p - 1, false);
  cy[1].build_ends(p, ne, s, p - 1, !(absorbing & WALL_BOTTOM), !(absorbing & WALL_TOP));
  return build_vector(ne, s, leaf);
}

int Plan::build_vector(int ne, int s, int leaf) {
  if (leaf <= 0) leaf = 8;
  leaf_size = leaf;
  for (int c = 0; c < 2; ++c)
    if (cx[c].n < 1 || cy[c].n < 1) return -1;
  cbase[0] = 0;
  cbase[1] = (int64_t)cx[0].n * cy[0].n;
  cbase[2] = cbase[1] + (int64_t)cx[1].n * cy[1].n;
  ndof = cbase[2];
  // the degree-p space of the x direction stands for the mesh (sp.ne, sp.s)
  sp = kind == SPACE_HDIV ? cx[0] : cx[1];
  n1d = sp.n;
  // coupled functions of space b for every function of space a: supports
  // overlapping on a set of positive length, a contiguous range (supports
  // ordered by their starts and ends)
  auto cross = [](const Space1D& a, const Space1D& b, std::vector<int>& lo, std::vector<int>& hi) {
    lo.assign(a.n, 0);
    hi.assign(a.n, -1);
    int k0 = 0;
    for (int i = 0; i < a.n; ++i) {
      while (k0 < b.n && b.sup1[k0] <= a.sup0[i]) ++k0;
      int k1 = k0;
      while (k1 < b.n && b.sup0[k1] < a.sup1[i]) ++k1;
      lo[i] = k0;
      hi[i] = k1 - 1;
    }
  };
  std::vector<int> xlo[2][2], xhi[2][2], ylo[2][2], yhi[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      cross(cx[a], cx[b], xlo[a][b], xhi[a][b]);
      cross(cy[a], cy[b], ylo[a][b], yhi[a][b]);
    }
  auto locate = [&](int64_t d, int& c, int& i, int& j) {
    c = d >= cbase[1] ? 1 : 0;
    const int64_t r = d - cbase[c];
    i = (int)(r % cx[c].n);
    j = (int)(r / cx[c].n);
  };
  rowptr.assign(ndof + 1, 0);
  for (int64_t d = 0; d < ndof; ++d) {
    int c, i, j;
    locate(d, c, i, j);
    int64_t cnt = 0;
    for (int b = 0; b < 2; ++b)
      cnt += (int64_t)std::max(0, xhi[c][b][i] - xlo[c][b][i] + 1) * std::max(0, yhi[c][b][j] - ylo[c][b][j] + 1);
    rowptr[d + 1] = rowptr[d] + cnt;
  }
  nnz = rowptr[ndof];
  if (nnz > (int64_t)0x7fffffff) return -1;
  col.assign(nnz, 0);
  for (int64_t d = 0; d < ndof; ++d) {
    int c, i, j;
    locate(d, c, i, j);
    int64_t q = rowptr[d];
    for (int b = 0; b < 2; ++b)   // component-major, then y, then x: increasing dof ids
      for (int jj = ylo[c][b][j]; jj <= yhi[c][b][j]; ++jj)
        for (int ii = xlo[c][b][i]; ii <= xhi[c][b][i]; ++ii) col[q++] = (int)(cbase[b] + (int64_t)jj * cx[b].n + ii);
  }
  return finish(ne, s, leaf,
                [&](int64_t d, int& x0, int& x1, int& y0, int& y1) {
                  int c, i, j;
                  locate(d, c, i, j);
                  x0 = cx[c].sup0[i]; x1 = cx[c].sup1[i]; y0 = cy[c].sup0[j]; y1 = cy[c].sup1[j];
                },
                [&](int64_t d, auto&& f) {
                  for (int64_t q = rowptr[d]; q < rowptr[d + 1]; ++q) f((int64_t)col[q]);
                });
}

void Plan::dof_support(int64_t d, int& x0, int& x1, int& y0, int& y1) const {
  if (kind == SPACE_H1) {
    const int n = sp.n, i = (int)(d % n), j = (int)(d / n);
    x0 = sp.sup0[i]; x1 = sp.sup1[i]; y0 = sp.sup0[j]; y1 = sp.sup1[j];
    return;
  }
  const int c = d >= cbase[1] ? 1 : 0;
  const int64_t r = d - cbase[c];
  const int i = (int)(r % cx[c].n), j = (int)(r / cx[c].n);
  x0 = cx[c].sup0[i]; x1 = cx[c].sup1[i]; y0 = cy[c].sup0[j]; y1 = cy[c].sup1[j];
}

int Plan::build_realform(const Plan& base) {
  if (base.ndof < 1 || base.nodes.empty() || base.kind == SPACE_REALFORM || (base.kind == SPACE_H1 && base.sp.n < 1))
    return -1;   // a forest has no single space
  kind = SPACE_REALFORM;
  sp = base.sp;
  leaf_size = base.leaf_size;
  // the same amalgamated tree: a node's own unknowns are twice its dofs
  amalg_group = base.amalg_group;
  amalg_max = base.amalg_max;
  amalg_own = 2 * base.amalg_own;
  n1d = base.n1d;
  ndof = 2 * base.ndof;
  if (ndof > (int64_t)0x3fffffff) return -1;
  // base's couplings of dof d, increasing
  std::vector<int64_t> nb_list;
  auto base_neighbours = [&](int64_t d) {
    nb_list.clear();
    if (!base.col.empty()) {
      for (int64_t q = base.rowptr[d]; q < base.rowptr[d + 1]; ++q) nb_list.push_back(base.col[q]);
      return;
    }
    const Space1D& S = base.sp;
    const int n = S.n, i = (int)(d % n), j = (int)(d / n);
    for (int jj = S.lo[j]; jj <= S.hi[j]; ++jj)
      for (int ii = S.lo[i]; ii <= S.hi[i]; ++ii) nb_list.push_back((int64_t)jj * n + ii);
  };
  rowptr.assign(ndof + 1, 0);
  for (int64_t d = 0; d < base.ndof; ++d) {
    const int64_t len = base.rowptr[d + 1] - base.rowptr[d];
    rowptr[2 * d + 1] = rowptr[2 * d] + 2 * len;
    rowptr[2 * d + 2] = rowptr[2 * d + 1] + 2 * len;
  }
  nnz = rowptr[ndof];
  if (nnz > (int64_t)0x7fffffff) return -1;
  col.assign(nnz, 0);
  for (int64_t d = 0; d < base.ndof; ++d) {
    base_neighbours(d);
    if ((int64_t)nb_list.size() * 2 != rowptr[2 * d + 1] - rowptr[2 * d]) return -1;
    int64_t q = rowptr[2 * d];
    for (int64_t j : nb_list) { col[q++] = (int)(2 * j); col[q++] = (int)(2 * j + 1); }
    std::copy(col.begin() + rowptr[2 * d], col.begin() + rowptr[2 * d + 1], col.begin() + rowptr[2 * d + 1]);
  }
  return finish(base.sp.ne, base.sp.s, leaf_size,
                [&](int64_t d, int& x0, int& x1, int& y0, int& y1) { base.dof_support(d / 2, x0, x1, y0, y1); },
                [&](int64_t d, auto&& f) {
                  for (int64_t q = rowptr[d]; q < rowptr[d + 1]; ++q) f((int64_t)col[q]);
                });
}

template <class Sup, class Nb>
int Plan::finish(int ne, int s, int leaf, Sup support, Nb neighbours) {
  // --- tree of boxes -------------------------------------------------------
  std::vector<Node> tmp;
  std::function<int(int, int, int, int)> make = [&](int x0, int x1, int y0, int y1) -> int {
    int id = (int)tmp.size();
    tmp.push_back(Node{});
    tmp[id].x0 = x0; tmp[id].x1 = x1; tmp[id].y0 = y0; tmp[id].y1 = y1;
    int cx = pick_cut(x0, x1, s, leaf), cy = pick_cut(y0, y1, s, leaf);
    int dir = -1, cut = -1;
    if (x1 - x0 >= y1 - y0) {
      if (cx >= 0) { dir = 0; cut = cx; } else if (cy >= 0) { dir = 1; cut = cy; }
    } else {
      if (cy >= 0) { dir = 1; cut = cy; } else if (cx >= 0) { dir = 0; cut = cx; }
    }
    tmp[id].dir = dir; tmp[id].cut = cut;
    if (dir >= 0) {
      int a, b;
      if (dir == 0) { a = make(x0, cut, y0, y1); b = make(cut, x1, y0, y1); }
      else          { a = make(x0, x1, y0, cut); b = make(x0, x1, cut, y1); }
      tmp[id].children = {a, b};
      tmp[a].parent = id; tmp[b].parent = id;
    }
    return id;
  };
  int root_tmp = make(0, ne, 0, ne);

  // postorder renumbering
  std::vector<int> order;
  std::function<void(int)> dfs = [&](int v) {
    for (int c : tmp[v].children) dfs(c);
    order.push_back(v);
  };
  dfs(root_tmp);
  std::vector<int> newid(tmp.size());
  for (size_t k = 0; k < order.size(); ++k) newid[order[k]] = (int)k;
  nodes.assign(tmp.size(), Node{});
  for (size_t k = 0; k < order.size(); ++k) {
    Node nd = tmp[order[k]];
    nd.parent = nd.parent >= 0 ? newid[nd.parent] : -1;
    for (int& c : nd.children) c = newid[c];
    nd.post = (int)k;
    nodes[k] = nd;
  }
  for (auto& nd : nodes) {
    nd.first_desc = nd.post;
    nd.height = 0;
    for (int c : nd.children) {
      nd.first_desc = std::min(nd.first_desc, nodes[c].first_desc);
      nd.height = std::max(nd.height, nodes[c].height + 1);
    }
  }
  const int root = (int)nodes.size() - 1;
  height = nodes[root].height + 1;

  // --- assign dofs -----------------------------------------------------------
  node_of_dof.assign(ndof, -1);
  for (int64_t d = 0; d < ndof; ++d) {
    int x0, x1, y0, y1;
    support(d, x0, x1, y0, y1);
    int v = root;
    for (;;) {
      const Node& nd = nodes[v];
      if (nd.dir < 0) break;
      int a0 = nd.dir == 0 ? x0 : y0;
      int a1 = nd.dir == 0 ? x1 : y1;
      if (a0 < nd.cut && nd.cut < a1) break;
      v = (a1 <= nd.cut) ? nd.children[0] : nd.children[1];
    }
    node_of_dof[d] = v;
    nodes[v].own.push_back((int)d);  // increasing dof id by construction
  }
  amalgamate();
  elim_pos.assign(ndof, -1);
  int64_t pos = 0;
  for (auto& nd : nodes)
    for (int d : nd.own) elim_pos[d] = pos++;

  // --- boundary sets ---------------------------------------------------------
  std::vector<int> stamp(ndof, -1);
  for (auto& nd : nodes) {
    std::vector<int> S;
    auto is_anc = [&](int w) {
      const Node& a = nodes[w];
      return a.post > nd.post && a.first_desc <= nd.post;
    };
    for (int c : nd.children)
      for (int g : nodes[c].bnd)
        if (node_of_dof[g] != nd.post && stamp[g] != nd.post) { stamp[g] = nd.post; S.push_back(g); }
    for (int d : nd.own) {
      neighbours((int64_t)d, [&](int64_t g64) {
        const int g = (int)g64;
        int w = node_of_dof[g];
        if (w != nd.post && is_anc(w) && stamp[g] != nd.post) { stamp[g] = nd.post; S.push_back(g); }
      });
    }
    std::sort(S.begin(), S.end(), [&](int a, int b) { return elim_pos[a] < elim_pos[b]; });
    nd.bnd = std::move(S);
  }

  // --- flatten -----------------------------------------------------------------
  const int nn = (int)nodes.size();
  nf.resize(nn); no.resize(nn); nb.resize(nn);
  loff.resize(nn); uoff.resize(nn); foff.resize(nn + 1);
  lsize = usize = 0;
  foff[0] = 0;
  flops_dense = 0; solve_bytes = 0;
  max_front = max_own = max_nb = 0;
  for (int v = 0; v < nn; ++v) {
    no[v] = (int)nodes[v].own.size();
    nb[v] = (int)nodes[v].bnd.size();
    nf[v] = no[v] + nb[v];
    loff[v] = lsize; lsize += (int64_t)nf[v] * no[v];
    uoff[v] = usize; usize += (int64_t)nb[v] * nb[v];
    foff[v + 1] = foff[v] + nf[v];
    max_front = std::max(max_front, nf[v]);
    max_own = std::max(max_own, no[v]);
    max_nb = std::max(max_nb, nb[v]);
    double o = no[v], b = nb[v];
    flops_dense += o * o * o / 3.0 + b * o * o + b * b * o;
    solve_bytes += 2.0 * 8.0 * (o * (o + 1) / 2 + b * o);
  }
  fdofs.resize(foff[nn]); fkey.resize(foff[nn]); fpos.resize(foff[nn]);
  for (int v = 0; v < nn; ++v) {
    int o = foff[v];
    std::vector<std::pair<int, int>> kp;
    int t = 0;
    for (int d : nodes[v].own) { fdofs[o + t] = d; kp.push_back({d, t}); ++t; }
    for (int d : nodes[v].bnd) { fdofs[o + t] = d; kp.push_back({d, t}); ++t; }
    std::sort(kp.begin(), kp.end());
    for (int k = 0; k < t; ++k) { fkey[o + k] = kp[k].first; fpos[o + k] = kp[k].second; }
  }
  coff.assign(nn + 1, 0);
  clist.clear();
  for (int v = 0; v < nn; ++v) {
    for (int c : nodes[v].children) clist.push_back(c);
    coff[v + 1] = (int)clist.size();
  }
  moff.assign(nn + 1, 0);
  maps.clear();
  std::vector<int> posmap(ndof, -1);
  for (int v = 0; v < nn; ++v) moff[v + 1] = moff[v] + nb[v];
  maps.resize(moff[nn]);
  for (int u = 0; u < nn; ++u) {
    for (int t = 0; t < nf[u]; ++t) posmap[fdofs[foff[u] + t]] = t;
    for (int c : nodes[u].children)
      for (int k = 0; k < nb[c]; ++k) {
        int pz = posmap[nodes[c].bnd[k]];
        if (pz < 0) return -2;  // bnd(c) must lie in the parent front
        maps[moff[c] + k] = pz;
      }
    for (int t = 0; t < nf[u]; ++t) posmap[fdofs[foff[u] + t]] = -1;
  }
  // levels by height
  level_off.assign(height + 1, 0);
  for (auto& nd : nodes) level_off[nd.height + 1]++;
  for (int h = 0; h < height; ++h) level_off[h + 1] += level_off[h];
  level_nodes.assign(nn, 0);
  std::vector<int> fill(level_off.begin(), level_off.end() - 1);
  for (auto& nd : nodes) level_nodes[fill[nd.height]++] = nd.post;
  return 0;
}

void Plan::merge(const std::vector<const Plan*>& parts, std::vector<int64_t>& dof_base,
                 std::vector<int>& node_base) {
  *this = Plan();
  const size_t np = parts.size();
  dof_base.assign(np + 1, 0);
  node_base.assign(np + 1, 0);
  std::vector<int64_t> nnz_base(np + 1, 0), l_base(np + 1, 0), u_base(np + 1, 0);
  std::vector<int> f_base(np + 1, 0), c_base(np + 1, 0), m_base(np + 1, 0);
  for (size_t k = 0; k < np; ++k) {
    const Plan& q = *parts[k];
    dof_base[k + 1] = dof_base[k] + q.ndof;
    node_base[k + 1] = node_base[k] + (int)q.nodes.size();
    nnz_base[k + 1] = nnz_base[k] + q.nnz;
    l_base[k + 1] = l_base[k] + q.lsize;
    u_base[k + 1] = u_base[k] + q.usize;
    f_base[k + 1] = f_base[k] + (int)q.fdofs.size();
    c_base[k + 1] = c_base[k] + (int)q.clist.size();
    m_base[k + 1] = m_base[k] + (int)q.maps.size();
  }
  ndof = dof_base[np];
  nnz = nnz_base[np];
  lsize = l_base[np];
  usize = u_base[np];
  const int nn = node_base[np];
  rowptr.assign(ndof + 1, 0);
  nodes.resize(nn);
  node_of_dof.assign(ndof, 0);
  elim_pos.assign(ndof, 0);
  nf.resize(nn); no.resize(nn); nb.resize(nn);
  loff.resize(nn); uoff.resize(nn);
  foff.assign(nn + 1, 0);
  fdofs.resize(f_base[np]); fkey.resize(f_base[np]); fpos.resize(f_base[np]);
  coff.assign(nn + 1, 0);
  clist.resize(c_base[np]);
  moff.assign(nn + 1, 0);
  maps.resize(m_base[np]);
  for (size_t k = 0; k < np; ++k) {
    const Plan& q = *parts[k];
    const int64_t db = dof_base[k];
    const int nbk = node_base[k];
    for (int64_t r = 0; r <= q.ndof; ++r) rowptr[db + r] = q.rowptr[r] + nnz_base[k];
    for (int64_t d = 0; d < q.ndof; ++d) {
      node_of_dof[db + d] = q.node_of_dof[d] + nbk;
      elim_pos[db + d] = q.elim_pos[d] + db;
    }
    for (size_t v = 0; v < q.nodes.size(); ++v) {
      Node nd = q.nodes[v];
      if (nd.parent >= 0) nd.parent += nbk;
      for (int& c : nd.children) c += nbk;
      for (int& d : nd.own) d += (int)db;
      for (int& d : nd.bnd) d += (int)db;
      nd.post += nbk;
      nd.first_desc += nbk;
      const int g = nbk + (int)v;
      nodes[g] = std::move(nd);
      nf[g] = q.nf[v]; no[g] = q.no[v]; nb[g] = q.nb[v];
      loff[g] = q.loff[v] + l_base[k];
      uoff[g] = q.uoff[v] + u_base[k];
      foff[g] = q.foff[v] + f_base[k];
      coff[g] = q.coff[v] + c_base[k];
      moff[g] = q.moff[v] + m_base[k];
    }
    for (size_t t = 0; t < q.fdofs.size(); ++t) {
      fdofs[f_base[k] + t] = q.fdofs[t] + (int)db;
      fkey[f_base[k] + t] = q.fkey[t] + (int)db;
      fpos[f_base[k] + t] = q.fpos[t];
    }
    for (size_t t = 0; t < q.clist.size(); ++t) clist[c_base[k] + t] = q.clist[t] + nbk;
    for (size_t t = 0; t < q.maps.size(); ++t) maps[m_base[k] + t] = q.maps[t];
    height = std::max(height, q.height);
    max_front = std::max(max_front, q.max_front);
    max_own = std::max(max_own, q.max_own);
    max_nb = std::max(max_nb, q.max_nb);
    flops_dense += q.flops_dense;
    solve_bytes += q.solve_bytes;
    if (q.sym_nnz_l < 0 || (k > 0 && sym_nnz_l < 0)) {
      sym_nnz_l = -1;
      sym_flops = -1.0;
    } else {
      sym_nnz_l = (k == 0 ? 0 : sym_nnz_l) + q.sym_nnz_l;
      sym_flops = (k == 0 ? 0.0 : sym_flops) + q.sym_flops;
    }
  }
  foff[nn] = f_base[np];
  coff[nn] = c_base[np];
  moff[nn] = m_base[np];
  level_off.assign(height + 1, 0);
  for (auto& nd : nodes) level_off[nd.height + 1]++;
  for (int h = 0; h < height; ++h) level_off[h + 1] += level_off[h];
  level_nodes.assign(nn, 0);
  std::vector<int> fill(level_off.begin(), level_off.end() - 1);
  for (auto& nd : nodes) level_nodes[fill[nd.height]++] = nd.post;
}

}  // namespace riga
