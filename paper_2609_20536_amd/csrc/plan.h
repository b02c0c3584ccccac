// Charge-block plans for the contractions of one HOTRG step.
//
// At h = h1 = 0 the site tensor conserves the U(1) charge
// q_l + q_d = q_r + q_u (Ch. 3: the field factor reduces to a Kronecker
// delta, and the thesis notes the resulting charge conservation); at h = 0,
// h1 != 0 only the parity of that sum survives (Z2); with h != 0 nothing.
// Every contraction of a step then splits into independent dense products,
// one per value of a conserved combination of leg charges (the block-sparse
// treatment of symmetric tensors the thesis recommends in the SVD section).
// A plan lists, per group, the element offsets of the rows, the reduction
// index and the columns of both operands and of the output; the grouped GEMM
// reads the tensors in place through these tables.
#pragma once

#include <map>
#include <vector>

#include "internal.h"

namespace gxy {

// Charge arithmetic: mod 0 = integers (U(1)), 2 = parities (Z2), 1 = trivial.
inline int qnorm(int x, int mod) {
  if (mod == 0) return x;
  if (mod == 1) return 0;
  return ((x % mod) + mod) % mod;
}

// Allowed values of Q = q_l + q_d - q_r - q_u of a tensor T[l][r][u][d].
typedef std::vector<int> QSet;

QSet qset_negate(const QSet &s, int mod);
QSet qset_sum(const QSet &a, const QSet &b, int mod);

struct Launch {
  int32_t first_group = 0, ngroups = 0, total_tiles = 0, tile = 64;
  bool kfast_a = false, nfast_b = false;
  bool contig = false;  // groups of contiguous ranges (GroupedGemm::contig)
  // symmetric groups: C = A A^T (M = N, the rows' and columns' tables the
  // same, B read through A's tables transposed); only the tiles on and below
  // the diagonal run, each off-diagonal one writing its transpose as well
  bool sym = false;
  double flops = 0.0;  // algorithmic 2 M N K summed over groups
  double bytes = 0.0;  // algorithmic FP64 bytes: A, B read once, C written once
  double c_bytes = 0.0;  // 8 M N over the groups: C read once more when beta != 0
};

struct TablePlan {
  std::vector<GGroup> groups;
  std::vector<int64_t> tab;
  void clear() {
    groups.clear();
    tab.clear();
  }
};

struct StepLegs {
  int Dh, Dv, Dn, mod;
  std::vector<int> lh, lv, ln;  // labels of l/r legs, u/d legs, new a/b legs
  int tile = 0;  // projection tiles: 0 = chosen by tile fill, else 64 or 128
  // Block order of a fused (horizontal h, vertical v) index: grouped by
  // kappa = q_h - q_v (ascending), then h, then v. pos[h * Dv + v] is the
  // position in that order; vrank[v] is v's rank among the vertical indices
  // of its label, so that pos(h, v) = pos(h, v0) + vrank[v] - vrank[v0] for
  // v, v0 of one label. Filled by block_positions.
  std::vector<int64_t> pos;
  std::vector<int32_t> vrank;
};

// Fills L.pos and L.vrank from the leg labels.
void block_positions(StepLegs &L);

// Environment Gram matrices of one side (right = false: E_L, else E_R):
// three launches (top Gram, bottom Gram, E). Output layouts as in the dense
// path: env [(x, i), (x', i')] with row length Dh*Dv; E [nf x nf].
void plan_env(const StepLegs &L, bool right, TablePlan &tp, Launch out[3]);

// Projection factors for output columns a in [a0, a1), with the fused
// (l2, i) and (r2, d) indices stored in block order (pos):
//  X[a-a0][r1][u][pos(l2,i)] = sum_l1 P[(l1,l2),a] A[l1][r1][u][i]    (A in sA)
//  Y[a-a0][r1][u][pos(r2,d)] = sum_(l2,i) X[..][pos(l2,i)] B2[pos(l2,i)][pos(r2,d)]
//  T'[a][b][u][d]     += alpha sum_(r1,r2) Y[a-a0][r1][u][pos(r2,d)] P[(r1,r2),b]
// with B2[pos(l2,i)][pos(r2,d)] = B[l2][r2][i][d] (B in sB). Every charge
// block of the D^7 product Y = X B2 then reads and writes contiguous rows.
// plan_proj_y takes at most one of sA, sB with several charges (each output
// block then has one reduction block); a product of two charged factors is
// planned once per charge of A and accumulated.
Launch plan_proj_x(const StepLegs &L, int a0, int a1, const QSet &sA, TablePlan &tp);
Launch plan_proj_y(const StepLegs &L, int a0, int a1, const QSet &sA, const QSet &sB,
                   TablePlan &tp);
Launch plan_proj_t(const StepLegs &L, int a0, int a1, const QSet &sY, TablePlan &tp);

}  // namespace gxy
