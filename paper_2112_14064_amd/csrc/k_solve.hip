// Forward and backward sweeps with the multifrontal factor (Sec. 5.2.2: one
// forward/backward elimination per Arnoldi step, line 8 of Alg. 2).
//
// The factorization leaves, per node, F = [L_oo^{-1}; L_bo L_oo^{-1}]
// (nf x no, column-major) and its transpose.  With the front vector f (own
// entries of the right-hand side plus the children's update vectors):
//   forward   y_own = L_oo^{-1} f_own,   upd_v = f_bnd - (L_bo L_oo^{-1}) f_own
//             i.e. one product F f_own;
//   backward  x_own = L_oo^{-T} (y_own - L_bo^T x_bnd)
//                   = L_oo^{-T} y_own - (L_bo L_oo^{-1})^T x_bnd
//             i.e. one product F^T [y_own; -x_bnd].
// Every node is therefore a single matrix-vector product with no dependency
// chain inside it; only the tree levels are sequential.  A node's rows are split
// into tasks of 64 rows (one workgroup each: lane = row, the 8 waves take
// interleaved chunks of column groups, partial sums combined in LDS); every
// load is a coalesced 16-byte load per lane (2 FP64 or 4 FP32 entries, from
// the packed layouts of the factorization) and up to 4 right-hand sides share
// it.  F may be stored in FP32 (mixed-precision factor): its entries are
// widened on load and every sum is accumulated in FP64.
// The forward pass gathers children's vectors instead of scattering into
// shared boundary entries, so neither sweep needs atomics and results are
// bitwise reproducible.
#include "kernels.hpp"

namespace riga {

constexpr int SR = 64;            // rows per task: one per lane
// Factor blocks are read in the sweep layouts written by the factorization:
// K = 16 bytes / element consecutive columns (forward) or rows (backward) of
// F side by side, one 16-byte load per lane and group.  Tile shape of a task
// (a template pair, chosen per tree level by the autotuner): NW waves share
// the columns of the task's 64 rows, each wave keeping SG group loads in
// flight per round.  sweep_variant() lists the compiled shapes.
template <class E>
struct Pack {
  static constexpr int K = 16 / sizeof(E);
  typedef E V __attribute__((ext_vector_type(K)));
};

// One round of a wave: SG group loads g0 .. g0 + SG - 1 of the lane's row
// (forward) or column (backward), at p[off(g)]: p is the lane's entry of group
// 0 and off(g) the group's offset, the same for every lane.  Groups past the
// end are clamped to the last group and groups the layout leaves out for a
// lane (their address then holds a neighbouring group's entries of the node)
// are masked in fma_round: the loads carry no branch, so the compiler can
// keep the next round in flight while the current one is used.
template <int SG, class V, class Off>
__device__ __forceinline__ void load_round(V (&a)[SG], const V* p, int g0, int gend, Off off) {
  const int glast = max(gend - 1, 0);
#pragma unroll
  for (int u = 0; u < SG; ++u) a[u] = p[off(min(g0 + u, glast))];
}

// acc[q] of row `lane` summed over the waves through LDS; wave 0 ends with the
// total for its lane.
template <int NR, int NW>
__device__ __forceinline__ void reduce_waves(double (&acc)[NR], double* red, int lane, int wave) {
#pragma unroll
  for (int q = 0; q < NR; ++q) red[(wave * SR + lane) * NR + q] = acc[q];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      double s2 = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) s2 += red[(w2 * SR + lane) * NR + q];
      acc[q] = s2;
    }
  }
}

// acc[q] += sum over the SG groups of a round (group g0 + u of the wave) of
// the K entries of each group times the LDS vector entries they multiply;
// groups at or past gend, or not stored for the lane (stored(g) false),
// contribute nothing.
template <int NR, int SG, int K, class V, class Stored>
__device__ __forceinline__ void fma_round(double (&acc)[NR], const V (&a)[SG], int g0, int gend,
                                          const double* vec, int nlast, Stored stored) {
#pragma unroll
  for (int u = 0; u < SG; ++u) {
    const bool in = g0 + u < gend && stored(g0 + u);
#pragma unroll
    for (int e = 0; e < K; ++e) {
      const int j = min((g0 + u) * K + e, nlast);
      const double av = in ? (double)a[u][e] : 0.0;
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[q] += av * vec[j * NR + q];
    }
  }
}

// Forward sweep of one level, one task (64 rows of F of a node) per workgroup.
// The factor does not depend on the front vector: two rounds of factor loads
// are in flight while the front is gathered, and rounds alternate between two
// register buffers so the next round is always loading.
template <int NR, class E, int NW, int SG>
__global__ __launch_bounds__(NW * 64) void k_fwd(DevTree t, const SweepTask* __restrict__ tasks,
                                            const E* __restrict__ Lp,
                                            const double* __restrict__ b, int64_t ldb,
                                            double* __restrict__ y, int64_t ldy,
                                            double* __restrict__ upd) {
  extern __shared__ double shm[];
  double* f = shm;                       // f[pos * NR + q], front vector
  const SweepTask tk = tasks[blockIdx.x];
  if (t.ilive != nullptr && !t.ilive[tk.inst]) return;
  const int r0 = tk.r0, r1 = tk.r1, nf = tk.nf, no = tk.no;
  double* red = shm + (size_t)nf * NR;   // NW x SR x NR partial sums
  const int* fd = t.fdofs + tk.foff;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = r0 + lane;
  const bool live = r < r1;
  // columns past the diagonal of L_oo^{-1} are exact zeros: an own-row block
  // stops at its last row's diagonal
  const int jend = (r1 - 1 < no) ? r1 : no;
  constexpr int K = Pack<E>::K;
  constexpr int STEP = NW * SG;
  typedef typename Pack<E>::V V;
  // group g of row r at lp[lp_group(g) + r - gK] for r >= gK (the rows above
  // are not stored: zeros of L_oo^{-1}); entries past the diagonal inside a
  // stored group are stored zeros
  // (32-bit offsets within the node: lp_group(g) - gK of kernels.hpp; a lane
  // above a group's first row reads the previous group's rows, masked)
  const int rr = live ? r : r0;
  const V* lp = reinterpret_cast<const V*>(Lp + tk.poff) + rr;
  auto at = [&](int g) { return g * nf - (K / 2) * g * (g - 1) - g * K; };
  auto stored = [&](int g) { return rr >= g * K; };
  const int gend = (jend + K - 1) / K;
  // front vector: own entries of b plus the children's update rows, added in
  // child order (one pass, no barrier per child).  A position's record
  // {dof or -1, update rows, first update row, second row or list start}
  // gives the b entry and up to two update rows in one load; the record of
  // the first gather round is requested before the factor, so that waiting
  // for it does not wait for the factor loads.  Only the positions the task
  // reads are gathered: the columns of its product, [0, nown), and its
  // boundary rows past them, [rb, r1).
  const int nown = min(nf, gend * K), rb = max(nown, r0);
  const int ng = nown + max(0, r1 - rb);
  const int4* gs = t.gsrc + tk.foff;
  const int4 rec0 = gs[min(tid < nown ? tid : rb + tid - nown, nf - 1)];
  __builtin_amdgcn_sched_barrier(0);      // keep the issue order
  int g = __builtin_amdgcn_readfirstlane(wave) * SG;
  V A[SG], B[SG];
  load_round<SG>(A, lp, g, gend, at);
  load_round<SG>(B, lp, g + STEP, gend, at);
  const int dst = fd[min(r, nf - 1)];      // used by own rows only

  for (int i = tid; i < ng; i += NW * 64) {
    const int p = i < nown ? i : rb + i - nown;
    const int4 rc = (i == tid) ? rec0 : gs[p];
    double s[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) s[q] = (rc.x >= 0) ? b[rc.x + q * ldb] : 0.0;
    if (rc.y > 0) {
      const double* uc = upd + (int64_t)rc.z * NR;
#pragma unroll
      for (int q = 0; q < NR; ++q) s[q] += uc[q];
      if (rc.y == 2) {
        const double* u2 = upd + (int64_t)rc.w * NR;
#pragma unroll
        for (int q = 0; q < NR; ++q) s[q] += u2[q];
      } else {
        for (int k = 1; k < rc.y; ++k) {
          const double* u2 = upd + (int64_t)t.gidx[rc.w + k] * NR;
#pragma unroll
          for (int q = 0; q < NR; ++q) s[q] += u2[q];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) f[p * NR + q] = s[q];
  }
  __syncthreads();
  double acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = 0.0;
  while (g < gend) {
    fma_round<NR, SG, K>(acc, A, g, gend, f, nown - 1, stored);
    load_round<SG>(A, lp, g + 2 * STEP, gend, at);
    g += STEP;
    if (g >= gend) break;
    fma_round<NR, SG, K>(acc, B, g, gend, f, nown - 1, stored);
    load_round<SG>(B, lp, g + 2 * STEP, gend, at);
    g += STEP;
  }
  reduce_waves<NR, NW>(acc, red, lane, wave);
  if (wave == 0 && live) {
    if (r < no) {
      // signed factor L S L^T: the backward sweep starts from S L^{-1} b
      const double sg = t.sgn != nullptr ? t.sgn[dst] : 1.0;
#pragma unroll
      for (int q = 0; q < NR; ++q) y[dst + q * ldy] = acc[q] * sg;
    } else {
      double* uv = upd + (int64_t)(tk.voff + r - no) * NR;
#pragma unroll
      for (int q = 0; q < NR; ++q) uv[q] = f[r * NR + q] - acc[q];
    }
  }
}

// Backward sweep of one level, one task (64 own columns of a node) per
// workgroup, loads pipelined as in the forward sweep.  The sweep's own result
// x (needed by the descendants as boundary values) is kept in xs, negated
// when `neg` is set.  Optional outputs: ru = scale (x + base) (base may be
// null; ru may alias base: each entry is read and written by one thread) and
// rl = sig val + v_u, where val is the ru value or, without ru, the xs value.
template <int NR, class E, int NW, int SG, bool TRI>
__global__ __launch_bounds__(NW * 64) void k_bwd(DevTree t, const SweepTask* __restrict__ tasks,
                                            const E* __restrict__ Tp,
                                            const double* __restrict__ y, int64_t ldy,
                                            double* __restrict__ xs, int64_t ldxs, int neg,
                                            const double* base, int64_t ldbase, double* ru, int64_t ldr,
                                            double scale,
                                            double* __restrict__ rl, const double* __restrict__ v_u,
                                            int64_t ldv, double sig) {
  extern __shared__ double shm[];
  double* w = shm;                       // [y_own; -x_bnd]
  const SweepTask tk = tasks[blockIdx.x];
  if (t.ilive != nullptr && !t.ilive[tk.inst]) return;
  const int a0 = tk.r0, a1 = tk.r1, nf = tk.nf, no = tk.no;
  double* red = shm + (size_t)nf * NR;
  const int* fd = t.fdofs + tk.foff;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int a = a0 + lane;
  const bool live = a < a1;
  constexpr int K = Pack<E>::K;
  constexpr int STEP = NW * SG;
  typedef typename Pack<E>::V V;
  // rows of F in groups of K: group g of own column a at tp[tp_group(g) + a]
  // for a < tp_width(g) (or at tp[g no + a] in the full rectangle); the groups
  // above the column's diagonal block are zeros, so the task starts at group
  // a0 / K.  Offsets are 32-bit within the node; a lane right of a group's
  // width reads the next group's columns, masked.  TRI: the level's nodes
  // leave out the zero triangle (launch_bwd_level), else the full rectangle.
  const int aa = live ? a : a0;
  const V* tp = reinterpret_cast<const V*>(Tp + tk.poff) + aa;
  // tp_group(g) = g no - (x no - K x (x + 1) / 2), x = min(g, g1 - 1): the
  // rectangle's offset less the columns the groups before g leave out;
  // straight-line scalar arithmetic (tri = 0: the full rectangle)
  const int g1m = (no + K - 1) / K - 1;
  auto at = [&](int g) {
    if (!TRI) return g * no;
    const int x = min(g, g1m);
    return g * no - (x * no - (K / 2) * x * (x + 1));
  };
  auto stored = [&](int g) { return !TRI || aa < (g + 1) * K; };
  const int gend = (nf + K - 1) / K;
  // indices of the first gather round before the factor loads (see k_fwd)
  const int fd0 = fd[min(tid, nf - 1)];
  __builtin_amdgcn_sched_barrier(0);      // keep the issue order
  int g = a0 / K + __builtin_amdgcn_readfirstlane(wave) * SG;
  V A[SG], B[SG];
  load_round<SG>(A, tp, g, gend, at);
  load_round<SG>(B, tp, g + STEP, gend, at);
  const int d = fd[min(a, no - 1)];       // used by live lanes only
  if (t.inst != nullptr) sig = t.isig[tk.inst];

  for (int p = tid; p < nf; p += NW * 64) {
    const int fp = (p == tid) ? fd0 : fd[p];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      double val;
      if (p < no) {
        val = y[fp + q * ldy];
      } else {
        val = xs[fp + q * ldxs];
        if (!neg) val = -val;
      }
      w[p * NR + q] = val;
    }
  }
  // the entries the epilogue adds are requested now: their latency passes
  // during the product
  double bpre[NR], vpre[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    bpre[q] = (wave == 0 && ru != nullptr && base != nullptr) ? base[d + q * ldbase] : 0.0;
    vpre[q] = (wave == 0 && rl != nullptr) ? v_u[d + q * ldv] : 0.0;
  }
  __syncthreads();
  double acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = 0.0;
  while (g < gend) {
    fma_round<NR, SG, K>(acc, A, g, gend, w, nf - 1, stored);
    load_round<SG>(A, tp, g + 2 * STEP, gend, at);
    g += STEP;
    if (g >= gend) break;
    fma_round<NR, SG, K>(acc, B, g, gend, w, nf - 1, stored);
    load_round<SG>(B, tp, g + 2 * STEP, gend, at);
    g += STEP;
  }
  reduce_waves<NR, NW>(acc, red, lane, wave);
  if (wave == 0 && live) {
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      double val = neg ? -acc[q] : acc[q];
      xs[d + q * ldxs] = val;
      if (ru != nullptr) {
        val = scale * (acc[q] + bpre[q]);
        ru[d + q * ldr] = val;
      }
      if (rl != nullptr) rl[d + q * ldr] = sig * val + vpre[q];
    }
  }
}

int sweep_variants() { return 8; }

void sweep_variant(int v, int* waves, int* groups) {
  static const int W[8] = {8, 8, 8, 4, 4, 4, 16, 16}, G[8] = {4, 2, 8, 4, 2, 8, 2, 1};
  *waves = W[v];
  *groups = G[v];
}

int sweep_default_variant(int tasks, bool forward) {
  // measured per level on the rIGA p=3 256^2 tree (8 levels), FP64, 2 right-hand sides
  if (tasks >= 1024) return 4;                 // 4 waves x 2 groups
  if (forward) return tasks >= 64 ? 1 : 7;     // 8 x 2, or 16 x 1
  return tasks >= 256 ? 1 : 6;                 // 8 x 2, or 16 x 2
}

namespace {

template <int NR, class E, int NW, int SG>
void fwd_one(const DevTree& t, const SweepTask* tasks, int count, const E* Lp, const double* b, int64_t ldb, double* y,
             int64_t ldy, double* upd, int max_front, hipStream_t st) {
  const size_t shm = ((size_t)max_front + NW * SR) * NR * sizeof(double);
  hipLaunchKernelGGL((k_fwd<NR, E, NW, SG>), dim3(count), dim3(NW * 64), shm, st, t, tasks, Lp, b, ldb, y, ldy, upd);
}

template <int NR, class E>
void fwd_shape(int variant, const DevTree& t, const SweepTask* tasks, int count, const E* Lp, const double* b,
               int64_t ldb, double* y, int64_t ldy, double* upd, int max_front, hipStream_t st) {
  switch (variant) {
    case 1: fwd_one<NR, E, 8, 2>(t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
    case 2: fwd_one<NR, E, 8, 8>(t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
    case 3: fwd_one<NR, E, 4, 4>(t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
    case 4: fwd_one<NR, E, 4, 2>(t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
    case 5: fwd_one<NR, E, 4, 8>(t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
    case 6: fwd_one<NR, E, 16, 2>(t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
    case 7: fwd_one<NR, E, 16, 1>(t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
    default: fwd_one<NR, E, 8, 4>(t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
  }
}

template <class E>
void fwd_nr(int nrhs, int variant, const DevTree& t, const SweepTask* tasks, int count, const E* Lp, const double* b,
            int64_t ldb, double* y, int64_t ldy, double* upd, int max_front, hipStream_t st) {
  switch (nrhs) {
    case 1: fwd_shape<1, E>(variant, t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
    case 2: fwd_shape<2, E>(variant, t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
    case 3: fwd_shape<3, E>(variant, t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
    default: fwd_shape<4, E>(variant, t, tasks, count, Lp, b, ldb, y, ldy, upd, max_front, st); break;
  }
}

template <int NR, class E, int NW, int SG>
void bwd_one(const DevTree& t, const SweepTask* tasks, int count, const E* Tp, const double* y, int64_t ldy,
             const BwdOut& o, int max_front, hipStream_t st) {
  const size_t shm = ((size_t)max_front + NW * SR) * NR * sizeof(double);
  // the level's layout: the rule of build_sweep_plan (its backward task count)
  if (count >= SWEEP_TRI_TASKS)
    hipLaunchKernelGGL((k_bwd<NR, E, NW, SG, true>), dim3(count), dim3(NW * 64), shm, st, t, tasks, Tp, y, ldy, o.xs,
                       o.ldxs, o.neg, o.base, o.ldbase, o.ru, o.ldr, o.scale, o.rl, o.v_u, o.ldv, o.sig);
  else
    hipLaunchKernelGGL((k_bwd<NR, E, NW, SG, false>), dim3(count), dim3(NW * 64), shm, st, t, tasks, Tp, y, ldy,
                       o.xs, o.ldxs, o.neg, o.base, o.ldbase, o.ru, o.ldr, o.scale, o.rl, o.v_u, o.ldv, o.sig);
}

template <int NR, class E>
void bwd_shape(int variant, const DevTree& t, const SweepTask* tasks, int count, const E* Tp, const double* y,
               int64_t ldy, const BwdOut& o, int max_front, hipStream_t st) {
  switch (variant) {
    case 1: bwd_one<NR, E, 8, 2>(t, tasks, count, Tp, y, ldy, o, max_front, st); break;
    case 2: bwd_one<NR, E, 8, 8>(t, tasks, count, Tp, y, ldy, o, max_front, st); break;
    case 3: bwd_one<NR, E, 4, 4>(t, tasks, count, Tp, y, ldy, o, max_front, st); break;
    case 4: bwd_one<NR, E, 4, 2>(t, tasks, count, Tp, y, ldy, o, max_front, st); break;
    case 5: bwd_one<NR, E, 4, 8>(t, tasks, count, Tp, y, ldy, o, max_front, st); break;
    case 6: bwd_one<NR, E, 16, 2>(t, tasks, count, Tp, y, ldy, o, max_front, st); break;
    case 7: bwd_one<NR, E, 16, 1>(t, tasks, count, Tp, y, ldy, o, max_front, st); break;
    default: bwd_one<NR, E, 8, 4>(t, tasks, count, Tp, y, ldy, o, max_front, st); break;
  }
}

template <class E>
void bwd_nr(int nrhs, int variant, const DevTree& t, const SweepTask* tasks, int count, const E* Tp, const double* y,
            int64_t ldy, const BwdOut& o, int max_front, hipStream_t st) {
  switch (nrhs) {
    case 1: bwd_shape<1, E>(variant, t, tasks, count, Tp, y, ldy, o, max_front, st); break;
    case 2: bwd_shape<2, E>(variant, t, tasks, count, Tp, y, ldy, o, max_front, st); break;
    case 3: bwd_shape<3, E>(variant, t, tasks, count, Tp, y, ldy, o, max_front, st); break;
    default: bwd_shape<4, E>(variant, t, tasks, count, Tp, y, ldy, o, max_front, st); break;
  }
}

}  // namespace

void launch_fwd_level(const DevTree& t, const SweepTask* tasks, int count, int nrhs, const double* Lp64,
                      const float* Lp32, const double* b, int64_t ldb, double* y, int64_t ldy, double* upd,
                      int max_front, int variant, hipStream_t st) {
  if (count <= 0) return;
  if (Lp32 != nullptr) fwd_nr<float>(nrhs, variant, t, tasks, count, Lp32, b, ldb, y, ldy, upd, max_front, st);
  else fwd_nr<double>(nrhs, variant, t, tasks, count, Lp64, b, ldb, y, ldy, upd, max_front, st);
}

void launch_bwd_level(const DevTree& t, const SweepTask* tasks, int count, int nrhs, const double* Tp64,
                      const float* Tp32, const double* y, int64_t ldy, const BwdOut& o, int max_front, int variant,
                      hipStream_t st) {
  if (count <= 0) return;
  if (Tp32 != nullptr) bwd_nr<float>(nrhs, variant, t, tasks, count, Tp32, y, ldy, o, max_front, st);
  else bwd_nr<double>(nrhs, variant, t, tasks, count, Tp64, y, ldy, o, max_front, st);
}

}  // namespace riga
