// Host-side symbolic plan: B-spline spaces, sparsity, nested-dissection tree
// whose separators are the rIGA hyperplanes, and the frontal index maps.
#pragma once
#include <cstdint>
#include <vector>

#ifndef RIGA_AMALG_GROUP
#define RIGA_AMALG_GROUP 2
#endif
#ifndef RIGA_AMALG_MAX
#define RIGA_AMALG_MAX 256
#endif
#ifndef RIGA_AMALG_OWN
#define RIGA_AMALG_OWN 640
#endif

namespace riga {

// One direction of the tensor-product space (Sec. 3.1).  Knot positions are
// kept as integers in element units: the open knot vector of eq. KnotsX with
// interior knots of multiplicity 1 (IGA, Sec. 3.2) or p at every s-th
// element boundary (rIGA with C^0 hyperplanes, Sec. 3.3).
struct Space1D {
  int p = 0, ne = 0, s = 0;
  int mult = 0;                // knot multiplicity at the hyperplanes
  int off = 1;                 // full index of function 0 (1: the end functions are removed)
  std::vector<int> knots;      // element-boundary indices 0..ne
  int nall = 0;                // functions before boundary elimination
  int n = 0;                   // functions kept: full indices off .. off + n - 1
  std::vector<int> sup0, sup1; // support [sup0, sup1) in elements, per kept function
  std::vector<int> lo, hi;     // coupled kept functions form the range [lo, hi]
  std::vector<int> first;      // per element: full index of its first nonzero function
  // mult_ < 0: p (C^0 hyperplanes); dirichlet: remove the first and last function
  void build(int p_, int ne_, int s_, int mult_ = -1, bool dirichlet = true);
  // the same with each end function removed or kept on its own
  void build_ends(int p_, int ne_, int s_, int mult_, bool drop_first, bool drop_last);
};

// Kinds of discrete space (riga_mesh.space).  SPACE_REALFORM is internal: the
// real form of a complex system on another plan's space (two unknowns per
// dof, see Plan::build_realform).
enum SpaceKind { SPACE_H1 = 0, SPACE_HCURL = 1, SPACE_HCURL_FREE = 2, SPACE_HDIV = 3, SPACE_REALFORM = 16 };
// Walls of the unit square (riga_mesh.walls, the absorbing ones of the
// divergence-conforming space).
enum Wall { WALL_LEFT = 1, WALL_RIGHT = 2, WALL_BOTTOM = 4, WALL_TOP = 8 };

struct Node {
  int x0, x1, y0, y1;          // box in element units
  int dir = -1, cut = -1;      // separator line: dir 0 -> x = cut, 1 -> y = cut, -1 leaf
  int parent = -1;
  std::vector<int> children;
  std::vector<int> own;        // dofs eliminated here, increasing dof id
  std::vector<int> bnd;        // ancestor dofs coupled to the subtree, elimination order
  int height = 0;
  int post = 0;                // postorder index
  int first_desc = 0;          // smallest postorder index in the subtree
};

struct Plan {
  Space1D sp;                  // identical in x and y (scalar space)
  int64_t n1d = 0, ndof = 0, nnz = 0;
  std::vector<int64_t> rowptr; // CSR row pointers of the tensor sparsity
  // Vector space (H(curl), Sec. 3.2 eq. HcurlBasis / Sec. 3.3): component c
  // has the tensor space cx[c] (x) cy[c], its dofs at cbase[c] + j n_x + i;
  // the CSR column indices are explicit (col).  Empty for the scalar space.
  int kind = SPACE_H1;
  int walls = 0;               // SPACE_HDIV: the absorbing walls (Wall bits)
  int leaf_size = 8;           // the leaf length the tree was built with
  Space1D cx[2], cy[2];
  int64_t cbase[3] = {0, 0, 0};
  std::vector<int> col;
  std::vector<Node> nodes;     // in postorder
  int height = 0;
  std::vector<int> level_nodes;    // node ids grouped by height
  std::vector<int> level_off;      // height h: level_nodes[level_off[h] .. level_off[h+1])
  std::vector<int> node_of_dof;
  std::vector<int64_t> elim_pos;   // dof -> elimination position
  // flattened frontal data
  std::vector<int> nf, no, nb;
  std::vector<int64_t> loff, uoff; // factor block (nf x no) and update block (nb x nb)
  int64_t lsize = 0, usize = 0;
  std::vector<int> foff;           // front dof list offsets
  std::vector<int> fdofs;          // front dofs: own then bnd
  std::vector<int> fkey, fpos;     // front dofs sorted by dof id, with their front positions
  std::vector<int> coff, clist;    // children (CSR)
  std::vector<int> moff, maps;     // per node: positions of its bnd dofs in the parent front
  int max_front = 0, max_own = 0, max_nb = 0;
  double flops_dense = 0.0;
  double solve_bytes = 0.0;

  // Amalgamation near the root: the depths holding at most amalg_max nodes
  // are taken amalg_group at a time, each group's top node absorbing the own
  // dofs of its descendants in the group (<= 1: off) when they number at most
  // amalg_own.  Those levels hold little data and the solve pays one
  // dependent step per level.
  int amalg_group = RIGA_AMALG_GROUP, amalg_max = RIGA_AMALG_MAX, amalg_own = RIGA_AMALG_OWN;

  int build(int p, int ne, int s, int leaf);  // 0 ok, <0 invalid
  // H(curl) space S^{p-1,p} x S^{p,p-1} (eq. HcurlBasis), rIGA hyperplanes of
  // multiplicity p-1 (C^1 in degree p, C^0 in degree p-1; eq.
  // DiscreteSpacesrIGA), every s elements; pec: tangential components vanish
  // on the boundary (the degree-p factor loses its end functions), else no
  // boundary condition.  p >= 2.
  int build_hcurl(int p, int ne, int s, int leaf, bool pec);
  // H(div) space S^{p,p-1} x S^{p-1,p} (eq. HdivBasis), the same hyperplanes;
  // a rigid wall (bit clear in `absorbing`) removes the degree-p function of
  // the normal direction that is nonzero on it (u.n = 0), an absorbing wall
  // keeps it.  p >= 2.
  int build_hdiv(int p, int ne, int s, int leaf, int absorbing);
  // The real form of a complex system on base's space: dof d of base becomes
  // the unknowns 2d (real part) and 2d + 1 (imaginary part), every coupling
  // of base a full 2 x 2 block; explicit columns; the same tree of boxes
  // (a dof's two unknowns are eliminated together).  Single-space bases only.
  int build_realform(const Plan& base);
  // Support box of a dof of a single-space plan, in elements.
  void dof_support(int64_t d, int& x0, int& x1, int& y0, int& y1) const;

  // Symbolic Cholesky of the tensor sparsity under the elimination order of
  // the plan (no dense-front zeros): per elimination position the nonzeros of
  // its column of L (diagonal included), their sum nnz(L), and the flops
  // sum_j (c_j^2 + 2 c_j) with c_j the off-diagonal count of column j.
  // Single-space plans only (a forest sums its parts' totals).
  void symbolic(std::vector<int64_t>* colcount, int64_t& nnz_l, double& flops) const;
  // Cached totals of symbolic() (computed on first use; a forest sets them
  // from its parts in merge()).
  int64_t sym_nnz_l = -1;
  double sym_flops = -1.0;
  void ensure_symbolic();

  // Forest of independent problems: the plans of `parts` side by side, with
  // dofs, CSR rows, nodes and factor blocks numbered consecutively (part k's
  // dofs start at dof_base[k], its nodes at node_base[k]) and tree levels
  // grouped by height across all parts.  The 1-D space stays empty.
  void merge(const std::vector<const Plan*>& parts, std::vector<int64_t>& dof_base,
             std::vector<int>& node_base);

 private:
  void amalgamate();
  // Tree, dof assignment, amalgamation, boundary sets and frontal data, given
  // ndof, rowptr and the dofs' supports and neighbours.
  template <class Sup, class Nb>
  int finish(int ne, int s, int leaf, Sup support, Nb neighbours);
  // vector space from its four component spaces (set in cx, cy) and kind
  int build_vector(int ne, int s, int leaf);
};

}  // namespace riga
