// Host check of the charge-block plans (no GPU): every table offset stays in
// bounds, and the grouped products, evaluated on the CPU through the offset
// tables exactly as the grouped GEMM reads them, equal the dense
// contractions of the environments and of the projection written out here
// (all three placements of the impurity chains, one and several chunks).

#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <random>
#include <vector>
#include "plan.h"
using namespace gxy;
static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { ++fails; if (fails < 20) { printf("FAIL %s:%d ", __FILE__, __LINE__); printf(__VA_ARGS__); printf("\n"); } } } while (0)

// emulate a launch: C = alpha A B + beta C, bounds-checked
void emulate(const TablePlan &tp, const Launch &L, const std::vector<double> &A, const std::vector<double> &B,
             std::vector<double> &C, double alpha, double beta, std::vector<int> *hits = nullptr) {
  for (int gi = 0; gi < L.ngroups; ++gi) {
    const GGroup &g = tp.groups[L.first_group + gi];
    auto T = [&](int64_t base, int i) { int64_t idx = base + i; CHECK(idx >= 0 && idx < (int64_t)tp.tab.size(), "tab idx"); return tp.tab[idx]; };
    // contiguous groups: rows through the table, k and n as ranges (GroupedGemm::contig)
    auto offA = [&](int m, int k) { return L.contig ? T(g.ar, m) + g.ac + k : T(g.ar, m) + T(g.ac, k); };
    auto offB = [&](int k, int n) { return L.contig ? g.br + (int64_t)k * g.bc + n : T(g.br, k) + T(g.bc, n); };
    auto offC = [&](int m, int n) { return L.contig ? T(g.ar, m) + g.cc + n : T(g.cr, m) + T(g.cc, n); };
    // symmetric launches (Launch::sym): only tiles on and below the diagonal
    // run; an off-diagonal one also writes the transposed element
    const int tsz = L.tile == 256 ? 128 : L.tile;
    CHECK(!L.sym || (g.M == g.N && L.tile != 256 && beta == 0.0), "sym launch shape");
    for (int m = 0; m < g.M; ++m) for (int n = 0; n < g.N; ++n) {
      if (L.sym && m / tsz < n / tsz) continue;
      const bool mirror = L.sym && m / tsz > n / tsz;
      double acc = 0;
      for (int k = 0; k < g.K; ++k) {
        int64_t ia = offA(m, k), ib = offB(k, n);
        CHECK(ia >= 0 && ia < (int64_t)A.size(), "A off %lld", (long long)ia);
        CHECK(ib >= 0 && ib < (int64_t)B.size(), "B off %lld", (long long)ib);
        if (ia >= 0 && ia < (int64_t)A.size() && ib >= 0 && ib < (int64_t)B.size()) acc += A[ia] * B[ib];
      }
      int64_t ic = offC(m, n);
      CHECK(ic >= 0 && ic < (int64_t)C.size(), "C off");
      if (ic >= 0 && ic < (int64_t)C.size()) {
        C[ic] = alpha * acc + (beta == 0.0 ? 0.0 : beta * C[ic]);
        if (hits) (*hits)[ic]++;
      }
      if (mirror) {
        int64_t it = offC(n, m);
        CHECK(it >= 0 && it < (int64_t)C.size(), "C off (mirror)");
        if (it >= 0 && it < (int64_t)C.size()) {
          C[it] = alpha * acc;
          if (hits) (*hits)[it]++;
        }
      }
    }
  }
}
int qn(int x, int mod) { return qnorm(x, mod); }
bool inS(int x, const QSet &s) { for (int v : s) if (v == x) return true; return false; }
// random tensor T[l][r][u][d] with Q = q_l + q_d - q_r - q_u in S
std::vector<double> rand_tensor(int Dh, int Dv, const std::vector<int> &lh, const std::vector<int> &lv, const QSet &S, int mod, std::mt19937 &rng) {
  std::normal_distribution<double> nd;
  std::vector<double> T((size_t)Dh*Dh*Dv*Dv, 0.0);
  for (int l = 0; l < Dh; ++l) for (int r = 0; r < Dh; ++r) for (int u = 0; u < Dv; ++u) for (int d = 0; d < Dv; ++d)
    if (inS(qn(lh[l] + lv[d] - lh[r] - lv[u], mod), S)) T[(((size_t)l*Dh + r)*Dv + u)*Dv + d] = nd(rng);
  return T;
}
void run_case(int Dh, int Dv, int Dn, int mod, int seed, const QSet &SX) {
  std::mt19937 rng(seed);
  std::uniform_int_distribution<int> ch(-3, 3);
  std::vector<int> lh(Dh), lv(Dv), ln(Dn);
  for (auto &x : lh) x = qn(ch(rng), mod);
  for (auto &x : lv) x = qn(ch(rng), mod);
  for (auto &x : ln) x = qn(ch(rng), mod);
  QSet s0{0};
  auto T = rand_tensor(Dh, Dv, lh, lv, s0, mod, rng);
  auto TX = rand_tensor(Dh, Dv, lh, lv, SX, mod, rng);
  const int64_t nf = (int64_t)Dh*Dh, MN = (int64_t)Dh*Dv, W = MN;
  // P: column a nonzero only for (l1,l2) with q_l1 + q_l2 = q_a
  std::normal_distribution<double> nd;
  std::vector<double> P(nf*Dn, 0.0);
  for (int l1 = 0; l1 < Dh; ++l1) for (int l2 = 0; l2 < Dh; ++l2) for (int a = 0; a < Dn; ++a)
    if (qn(lh[l1] + lh[l2], mod) == ln[a]) P[((int64_t)l1*Dh + l2)*Dn + a] = nd(rng);
  StepLegs SL{Dh, Dv, Dn, mod, lh, lv, ln};
  block_positions(SL);
  { std::vector<int> seen(W, 0); bool ok = true; for (int64_t x : SL.pos) { if (x < 0 || x >= W || seen[x]++) ok = false; } CHECK(ok, "pos is not a permutation"); }
  // ---- environments vs dense
  for (int right = 0; right < 2; ++right) {
    TablePlan tp; Launch L[3]; plan_env(SL, right, tp, L);
    std::vector<double> eA(MN*MN, NAN), eB(MN*MN, NAN), E(nf*nf, NAN);
    emulate(tp, L[0], T, T, eA, 1, 0); emulate(tp, L[1], T, T, eB, 1, 0); emulate(tp, L[2], eA, eB, E, 1, 0);
    auto t = [&](int l, int r, int u, int d) { return T[(((size_t)l*Dh + r)*Dv + u)*Dv + d]; };
    double maxerr = 0; int checked = 0;
    for (int x1 = 0; x1 < Dh; ++x1) for (int x2 = 0; x2 < Dh; ++x2) for (int y1 = 0; y1 < Dh; ++y1) for (int y2 = 0; y2 < Dh; ++y2) {
      if (qn(lh[x1] + lh[x2], mod) != qn(lh[y1] + lh[y2], mod)) continue;  // sector entries only
      double ref = 0;
      for (int o1 = 0; o1 < Dh; ++o1) for (int o2 = 0; o2 < Dh; ++o2) for (int u = 0; u < Dv; ++u) for (int d = 0; d < Dv; ++d) {
        double m1 = 0, m2 = 0;
        for (int i = 0; i < Dv; ++i) {
          if (!right) { m1 += t(x1,o1,u,i)*t(x2,o2,i,d); m2 += t(y1,o1,u,i)*t(y2,o2,i,d); }
          else { m1 += t(o1,x1,u,i)*t(o2,x2,i,d); m2 += t(o1,y1,u,i)*t(o2,y2,i,d); }
        }
        ref += m1*m2;
      }
      double got = E[(x1*Dh + x2)*nf + y1*Dh + y2];
      maxerr = std::max(maxerr, std::fabs(got - ref)); ++checked;
    }
    CHECK(maxerr < 1e-9, "env right=%d maxerr %g", right, maxerr);
    printf("env right=%d checked %d maxerr %.2e groups %d+%d+%d\n", right, checked, maxerr, L[0].ngroups, L[1].ngroups, L[2].ngroups);
  }
  // ---- projection vs dense: T'[a,b,u,d] = sum P P A B
  auto proj_ref = [&](const std::vector<double> &A, const std::vector<double> &B) {
    std::vector<double> R((size_t)Dn*Dn*Dv*Dv, 0.0);
    for (int a = 0; a < Dn; ++a) for (int bb = 0; bb < Dn; ++bb) for (int u = 0; u < Dv; ++u) for (int d = 0; d < Dv; ++d) {
      double acc = 0;
      for (int l1 = 0; l1 < Dh; ++l1) for (int l2 = 0; l2 < Dh; ++l2) { double pa = P[((int64_t)l1*Dh + l2)*Dn + a]; if (pa == 0) continue;
        for (int r1 = 0; r1 < Dh; ++r1) for (int r2 = 0; r2 < Dh; ++r2) { double pb = P[((int64_t)r1*Dh + r2)*Dn + bb]; if (pb == 0) continue;
          for (int i = 0; i < Dv; ++i) acc += pa*pb*A[(((size_t)l1*Dh + r1)*Dv + u)*Dv + i]*B[(((size_t)l2*Dh + r2)*Dv + i)*Dv + d]; } }
      R[(((size_t)a*Dn + bb)*Dv + u)*Dv + d] = acc;
    }
    return R;
  };
  auto swap_mid = [&](const std::vector<double> &B) { std::vector<double> o(B.size());
    for (int l2 = 0; l2 < Dh; ++l2) for (int r2 = 0; r2 < Dh; ++r2) for (int i = 0; i < Dv; ++i) for (int d = 0; d < Dv; ++d)
      o[(size_t)SL.pos[(size_t)l2*Dv + i]*W + SL.pos[(size_t)r2*Dv + d]] = B[(((size_t)l2*Dh + r2)*Dv + i)*Dv + d]; return o; };
  for (int chunk : {Dn, (Dn + 1)/2, 1}) {
    for (int variant = 0; variant < 4; ++variant) {
      // 0: T T, 1: T TX, 2: TX T, 3: TX TX (split by the charge of A)
      const std::vector<double> &A = (variant >= 2) ? TX : T;
      const std::vector<double> &B = (variant == 1 || variant == 3) ? TX : T;
      QSet sA = (variant >= 2) ? SX : s0, sB = (variant == 1 || variant == 3) ? SX : s0, sY = qset_sum(sA, sB, mod);
      auto B2 = swap_mid(B);
      std::vector<double> Tn((size_t)Dn*Dn*Dv*Dv, 0.0);
      for (int a0 = 0; a0 < Dn; a0 += chunk) {
        int a1 = std::min(Dn, a0 + chunk);
        TablePlan tp;
        Launch lx = plan_proj_x(SL, a0, a1, sA, tp), lt = plan_proj_t(SL, a0, a1, sY, tp);
        std::vector<double> X((size_t)(a1-a0)*W*W, NAN), Y((size_t)(a1-a0)*W*W, NAN);
        emulate(tp, lx, P, A, X, 1, 0);
        if (variant == 3 && sA.size() > 1 && sB.size() > 1) {
          // the blocks are first cleared by a product that writes every one
          // of them (as the engine's first Y launch of a chain does), then
          // each charge of A adds its part
          std::fill(Y.begin(), Y.end(), 0.0);
          for (int c : sA) {
            Launch ly = plan_proj_y(SL, a0, a1, QSet{c}, sB, tp);
            emulate(tp, ly, X, B2, Y, 1, 1);
          }
        } else {
          Launch ly = plan_proj_y(SL, a0, a1, sA, sB, tp);
          emulate(tp, ly, X, B2, Y, 1, 0);
        }
        emulate(tp, lt, Y, P, Tn, 1, 0);
      }
      auto R = proj_ref(A, B);
      double maxerr = 0; for (size_t e = 0; e < R.size(); ++e) maxerr = std::max(maxerr, std::fabs(R[e] - Tn[e]));
      CHECK(maxerr < 1e-9, "proj variant %d chunk %d maxerr %g", variant, chunk, maxerr);
      printf("proj variant %d chunk %d maxerr %.2e\n", variant, chunk, maxerr);
    }
  }
}
int main() {
  run_case(4, 3, 5, 0, 1, QSet{-1, 1});
  run_case(5, 4, 7, 0, 2, QSet{-2, 2});
  run_case(3, 5, 6, 2, 3, QSet{1});
  run_case(4, 4, 5, 2, 4, QSet{0});
  run_case(3, 3, 4, 1, 5, QSet{0});
  printf("fails %d\n", fails);
  return fails ? 1 : 0;
}
