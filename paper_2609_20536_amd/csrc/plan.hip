// Charge-block plans: host-side enumeration of the groups and offset tables
// of the grouped GEMM launches of one HOTRG step (see plan.h).
#include "plan.h"

#include <algorithm>
#include <utility>

namespace gxy {

void block_positions(StepLegs &L) {
  const int Dh = L.Dh, Dv = L.Dv;
  L.pos.assign((size_t)Dh * Dv, 0);
  L.vrank.assign(Dv, 0);
  std::map<int, int> seen;
  for (int v = 0; v < Dv; ++v) L.vrank[v] = seen[qnorm(L.lv[v], L.mod)]++;
  std::map<int, std::vector<int64_t>> by_kappa;   // fused h * Dv + v, h then v
  for (int h = 0; h < Dh; ++h)
    for (int v = 0; v < Dv; ++v) by_kappa[qnorm(L.lh[h] - L.lv[v], L.mod)].push_back((int64_t)h * Dv + v);
  int64_t at = 0;
  for (const auto &kv : by_kappa)
    for (int64_t f : kv.second) L.pos[f] = at++;
}

QSet qset_negate(const QSet &s, int mod) {
  QSet o;
  for (int x : s) o.push_back(qnorm(-x, mod));
  std::sort(o.begin(), o.end());
  o.erase(std::unique(o.begin(), o.end()), o.end());
  return o;
}

QSet qset_sum(const QSet &a, const QSet &b, int mod) {
  QSet o;
  for (int x : a)
    for (int y : b) o.push_back(qnorm(x + y, mod));
  std::sort(o.begin(), o.end());
  o.erase(std::unique(o.begin(), o.end()), o.end());
  return o;
}

namespace {

typedef std::pair<int, int> PI;
typedef std::map<int, std::vector<PI>> PairBuckets;

// (x, y) pairs grouped by qnorm(sx q[x] + sy q[y]); x outer, y inner.
PairBuckets pair_buckets(const std::vector<int> &qx, const std::vector<int> &qy, int sx, int sy,
                         int mod) {
  PairBuckets out;
  for (int x = 0; x < (int)qx.size(); ++x)
    for (int y = 0; y < (int)qy.size(); ++y)
      out[qnorm(sx * qx[x] + sy * qy[y], mod)].push_back(PI(x, y));
  return out;
}

std::map<int, std::vector<int>> leg_buckets(const std::vector<int> &q, int mod) {
  std::map<int, std::vector<int>> out;
  for (int i = 0; i < (int)q.size(); ++i) out[qnorm(q[i], mod)].push_back(i);
  return out;
}

bool in_set(int x, const QSet &s) { return std::find(s.begin(), s.end(), x) != s.end(); }

struct GSpec {
  int32_t M, N, K;
  int64_t ar, ac, br, bc, cr, cc;
};

int64_t put(TablePlan &tp, const std::vector<int64_t> &v) {
  const int64_t at = (int64_t)tp.tab.size();
  tp.tab.insert(tp.tab.end(), v.begin(), v.end());
  return at;
}

int choose_tile(const std::vector<GSpec> &gs) {
  int64_t t128 = 0;
  double work = 0.0;
  for (const auto &g : gs) {
    t128 += (int64_t)((g.M + 127) / 128) * ((g.N + 127) / 128);
    work += (double)g.M * g.N;
  }
  if (t128 < 256) return 64;
  return work / ((double)t128 * 128.0 * 128.0) >= 0.6 ? 128 : 64;
}

Launch finish_launch(TablePlan &tp, const std::vector<GSpec> &gs, bool kfa, bool nfb,
                     int force_tile = 0, bool contig = false, bool sym = false) {
  Launch L;
  L.first_group = (int32_t)tp.groups.size();
  L.kfast_a = kfa;
  L.nfast_b = nfb;
  L.contig = contig;
  L.sym = sym;
  L.tile = force_tile ? force_tile : choose_tile(gs);
  if (sym && tile_rows(L.tile) != tile_cols(L.tile))
    fail(GXY_EDEVICE, "symmetric launch needs square tiles");
  for (const auto &g : gs) {
    if (g.M <= 0 || g.N <= 0) continue;
    GGroup G;
    G.M = g.M;
    G.N = g.N;
    G.K = g.K;
    G.tile_start = L.total_tiles;
    G.ar = g.ar;
    G.ac = g.ac;
    G.br = g.br;
    G.bc = g.bc;
    G.cr = g.cr;
    G.cc = g.cc;
    const int tm = tile_rows(L.tile), tn = tile_cols(L.tile);
    if (sym) {
      if (g.M != g.N || g.ar != g.bc || g.ac != g.br)
        fail(GXY_EDEVICE, "symmetric launch: a group is not C = A A^T");
      const int64_t t = (g.M + tm - 1) / tm;
      L.total_tiles += (int32_t)(t * (t + 1) / 2);
    } else {
      L.total_tiles += ((g.M + tm - 1) / tm) * ((g.N + tn - 1) / tn);
    }
    L.flops += 2.0 * g.M * g.N * (double)g.K;
    L.bytes += 8.0 * ((double)g.M * g.K + (double)g.K * g.N + (double)g.M * g.N);
    L.c_bytes += 8.0 * (double)g.M * g.N;
    tp.groups.push_back(G);
    ++L.ngroups;
  }
  return L;
}

}  // namespace

void plan_env(const StepLegs &S, bool right, TablePlan &tp, Launch out[3]) {
  const int Dh = S.Dh, Dv = S.Dv, mod = S.mod;
  const int64_t sl = (int64_t)Dh * Dv * Dv, sr = (int64_t)Dv * Dv, MN = (int64_t)Dh * Dv;
  const int64_t nf = (int64_t)Dh * Dh;
  // --- top Gram: rows (x, i), reduction (y, u) with x the open horizontal
  // leg and y the contracted one.  left: x = l1, y = r1, key q_l1 + q_i =
  // q_r1 + q_u.  right: x = r1, y = l1, key q_r1 - q_i = q_l1 - q_u.
  {
    const PairBuckets rows = right ? pair_buckets(S.lh, S.lv, 1, -1, mod)
                                   : pair_buckets(S.lh, S.lv, 1, 1, mod);
    const PairBuckets ks = right ? pair_buckets(S.lh, S.lv, 1, -1, mod)
                                 : pair_buckets(S.lh, S.lv, 1, 1, mod);
    const int64_t sx = right ? sr : sl, sy = right ? sl : sr;
    std::vector<GSpec> gs;
    for (const auto &kv : rows) {
      std::vector<int64_t> ar, ac, cr, cc;
      for (const PI &p : kv.second) {
        ar.push_back(p.first * sx + p.second);
        cr.push_back((p.first * (int64_t)Dv + p.second) * MN);
        cc.push_back(p.first * (int64_t)Dv + p.second);
      }
      auto it = ks.find(kv.first);
      if (it != ks.end())
        for (const PI &p : it->second) ac.push_back(p.first * sy + p.second * (int64_t)Dv);
      GSpec g;
      g.M = g.N = (int32_t)ar.size();
      g.K = (int32_t)ac.size();
      g.ar = put(tp, ar);
      g.bc = g.ar;
      g.ac = put(tp, ac);
      g.br = g.ac;
      g.cr = put(tp, cr);
      g.cc = put(tp, cc);
      gs.push_back(g);
    }
    // (C = A A^T: the output rows and columns are the same pairs, placed
    // by cr and cc from one list)
    out[0] = finish_launch(tp, gs, false, true, 0, false, true);
  }
  // --- bottom Gram: rows (x, i), reduction (y, d).  left: x = l2, y = r2,
  // key q_l2 - q_i = q_r2 - q_d.  right: x = r2, y = l2, key q_r2 + q_i =
  // q_l2 + q_d.
  {
    const PairBuckets rows = right ? pair_buckets(S.lh, S.lv, 1, 1, mod)
                                   : pair_buckets(S.lh, S.lv, 1, -1, mod);
    const PairBuckets ks = right ? pair_buckets(S.lh, S.lv, 1, 1, mod)
                                 : pair_buckets(S.lh, S.lv, 1, -1, mod);
    const int64_t sx = right ? sr : sl, sy = right ? sl : sr;
    std::vector<GSpec> gs;
    for (const auto &kv : rows) {
      std::vector<int64_t> ar, ac, cr, cc;
      for (const PI &p : kv.second) {
        ar.push_back(p.first * sx + p.second * (int64_t)Dv);
        cr.push_back((p.first * (int64_t)Dv + p.second) * MN);
        cc.push_back(p.first * (int64_t)Dv + p.second);
      }
      auto it = ks.find(kv.first);
      if (it != ks.end())
        for (const PI &p : it->second) ac.push_back(p.first * sy + p.second);
      GSpec g;
      g.M = g.N = (int32_t)ar.size();
      g.K = (int32_t)ac.size();
      g.ar = put(tp, ar);
      g.bc = g.ar;
      g.ac = put(tp, ac);
      g.br = g.ac;
      g.cr = put(tp, cr);
      g.cc = put(tp, cc);
      gs.push_back(g);
    }
    out[1] = finish_launch(tp, gs, true, false, 0, false, true);
  }
  // --- E[(x1,x2),(x1',x2')] = sum_{i,i'} envA[x1,i,x1',i'] envB[x2,i,x2',i']
  // kappa = q_i - q_i'.  left: rows (l1,l1') with q_l1' - q_l1 = kappa, cols
  // (l2,l2') with q_l2 - q_l2' = kappa.  right: rows (r1,r1') with
  // q_r1 - q_r1' = kappa, cols (r2,r2') with q_r2' - q_r2 = kappa.
  {
    const PairBuckets rows = right ? pair_buckets(S.lh, S.lh, 1, -1, mod)
                                   : pair_buckets(S.lh, S.lh, -1, 1, mod);
    const PairBuckets cols = right ? pair_buckets(S.lh, S.lh, -1, 1, mod)
                                   : pair_buckets(S.lh, S.lh, 1, -1, mod);
    const PairBuckets ks = pair_buckets(S.lv, S.lv, 1, -1, mod);
    const int64_t row = (int64_t)Dv * MN;
    std::vector<GSpec> gs;
    for (const auto &kv : rows) {
      auto ic = cols.find(kv.first);
      if (ic == cols.end()) continue;
      std::vector<int64_t> ar, ac, bc, cr, cc;
      for (const PI &p : kv.second) {
        ar.push_back(p.first * row + p.second * (int64_t)Dv);
        cr.push_back(p.first * (int64_t)Dh * nf + p.second * (int64_t)Dh);
      }
      for (const PI &p : ic->second) {
        bc.push_back(p.first * row + p.second * (int64_t)Dv);
        cc.push_back(p.first * nf + p.second);
      }
      auto ik = ks.find(kv.first);
      if (ik != ks.end())
        for (const PI &p : ik->second) ac.push_back(p.first * MN + p.second);
      GSpec g;
      g.M = (int32_t)ar.size();
      g.N = (int32_t)bc.size();
      g.K = (int32_t)ac.size();
      g.ar = put(tp, ar);
      g.ac = put(tp, ac);
      g.br = g.ac;
      g.bc = put(tp, bc);
      g.cr = put(tp, cr);
      g.cc = put(tp, cc);
      gs.push_back(g);
    }
    out[2] = finish_launch(tp, gs, true, false);
  }
}

namespace {

// Distinct normalised labels of one leg (ascending) with their indices
// (ascending); slot[i] is the position of i's label in that list.
struct LegLabels {
  std::vector<int> q;
  std::vector<std::vector<int>> members;
};

LegLabels leg_labels(const std::vector<int> &lab, int mod) {
  LegLabels L;
  for (int x : lab) L.q.push_back(qnorm(x, mod));
  std::sort(L.q.begin(), L.q.end());
  L.q.erase(std::unique(L.q.begin(), L.q.end()), L.q.end());
  L.members.resize(L.q.size());
  for (int i = 0; i < (int)lab.size(); ++i) {
    const int s = (int)(std::lower_bound(L.q.begin(), L.q.end(), qnorm(lab[i], mod)) - L.q.begin());
    L.members[s].push_back(i);
  }
  return L;
}

// Offset lists keyed by (integer key in [lo, hi], label slot), stored flat
// (one array per list kind, slot s spanning [start[s], start[s + 1])):
// filled by a counting pass and a filling pass that visit the entries in
// the same order, so each slot keeps the order in which its entries were
// produced.
struct FlatLists {
  int lo = 0, nk = 0, nl = 0;
  std::vector<int64_t> start, first, second;
  FlatLists(int lo_, int hi_, int nl_) : lo(lo_), nk(hi_ - lo_ + 1), nl(nl_) {
    if (nk < 0) nk = 0;
    start.assign((size_t)nk * nl + 1, 0);
  }
  int at(int key, int slot) const {
    return (key < lo || key >= lo + nk) ? -1 : (key - lo) * nl + slot;
  }
  int64_t size(int s) const { return s < 0 ? 0 : start[s + 1] - start[s]; }
  // after the counts are in start[s + 1]: offsets, storage, fill cursors
  std::vector<int64_t> finish_counts() {
    for (size_t s = 1; s < start.size(); ++s) start[s] += start[s - 1];
    first.resize(start.back());
    second.resize(start.back());
    return std::vector<int64_t>(start.begin(), start.end() - 1);
  }
};

// Appends [b, e) to the table and returns where it starts.
int64_t put_range(TablePlan &tp, const int64_t *b, const int64_t *e) {
  const int64_t at = (int64_t)tp.tab.size();
  tp.tab.insert(tp.tab.end(), b, e);
  return at;
}

}  // namespace

Launch plan_proj_x(const StepLegs &S, int a0, int a1, const QSet &sA, TablePlan &tp) {
  const int Dh = S.Dh, Dv = S.Dv, Dn = S.Dn, mod = S.mod;
  const int64_t W = (int64_t)Dh * Dv, per_a = W * W;
  const auto l1s = leg_buckets(S.lh, mod);
  // rows (a, l2) keyed by c = q_a - q_l2 (= q_l1); a varies fastest
  std::map<int, std::vector<PI>> rows;
  for (int l2 = 0; l2 < Dh; ++l2)
    for (int a = a0; a < a1; ++a) rows[qnorm(S.ln[a] - S.lh[l2], mod)].push_back(PI(a, l2));
  // columns (r1, u, i) keyed by (kc = q_r1 + q_u - q_i, label of i); group
  // (c, label) takes the columns with c - kc in sA. With the label of i
  // fixed, the output offset splits into a row part (pos of (l2, first i of
  // the label)) and a column part (r1, u, rank of i in its label).
  const LegLabels V = leg_labels(S.lv, mod);
  const int nl = (int)V.q.size();
  int lo = 0, hi = -1;
  for (int r1 = 0; r1 < Dh; ++r1)
    for (int u = 0; u < Dv; ++u)
      for (int li = 0; li < nl; ++li) {
        const int k = qnorm(S.lh[r1] + S.lv[u] - V.q[li], mod);
        if (hi < lo) lo = hi = k;
        lo = std::min(lo, k);
        hi = std::max(hi, k);
      }
  FlatLists cols(lo, hi, nl);
  for (int r1 = 0; r1 < Dh; ++r1)
    for (int u = 0; u < Dv; ++u)
      for (int li = 0; li < nl; ++li)
        cols.start[cols.at(qnorm(S.lh[r1] + S.lv[u] - V.q[li], mod), li) + 1] +=
            (int64_t)V.members[li].size();
  std::vector<int64_t> cur = cols.finish_counts();
  for (int r1 = 0; r1 < Dh; ++r1)
    for (int u = 0; u < Dv; ++u)
      for (int li = 0; li < nl; ++li) {
        int64_t &c = cur[cols.at(qnorm(S.lh[r1] + S.lv[u] - V.q[li], mod), li)];
        for (int i : V.members[li]) {
          cols.first[c] = (int64_t)r1 * Dv * Dv + (int64_t)u * Dv + i;
          cols.second[c] = (int64_t)r1 * Dv * W + (int64_t)u * W + S.vrank[i];
          ++c;
        }
      }
  // table size of the groups below, so the table grows once
  int64_t total = 0;
  for (const auto &kv : rows) {
    const int c = kv.first;
    auto il = l1s.find(c);
    const int64_t nk1 = il != l1s.end() ? (int64_t)il->second.size() : 0;
    for (int li = 0; li < nl; ++li) {
      int64_t nc = 0;
      for (int sv : sA) nc += cols.size(cols.at(qnorm(c - sv, mod), li));
      if (nc) total += 2 * (int64_t)kv.second.size() + 2 * nk1 + 2 * nc;
    }
  }
  tp.tab.reserve(tp.tab.size() + total);
  std::vector<GSpec> gs;
  for (const auto &kv : rows) {
    const int c = kv.first;
    std::vector<int64_t> ar, ac, br;
    for (const PI &p : kv.second) ar.push_back((int64_t)p.second * Dn + p.first);
    auto il = l1s.find(c);
    if (il != l1s.end())
      for (int l1 : il->second) {
        ac.push_back((int64_t)l1 * Dh * Dn);
        br.push_back((int64_t)l1 * Dh * Dv * Dv);
      }
    for (int li = 0; li < nl; ++li) {
      const int i0 = V.members[li][0];
      int64_t nc = 0;
      for (int sv : sA) nc += cols.size(cols.at(qnorm(c - sv, mod), li));
      if (nc == 0) continue;
      GSpec g;
      g.M = (int32_t)ar.size();
      g.N = (int32_t)nc;
      g.K = (int32_t)ac.size();
      g.ar = put(tp, ar);
      g.ac = put(tp, ac);
      g.br = put(tp, br);
      g.bc = (int64_t)tp.tab.size();
      for (int sv : sA) {
        const int at = cols.at(qnorm(c - sv, mod), li);
        if (at >= 0)
          put_range(tp, cols.first.data() + cols.start[at], cols.first.data() + cols.start[at + 1]);
      }
      g.cr = (int64_t)tp.tab.size();
      for (const PI &p : kv.second)
        tp.tab.push_back((int64_t)(p.first - a0) * per_a + S.pos[(size_t)p.second * Dv + i0]);
      g.cc = (int64_t)tp.tab.size();
      for (int sv : sA) {
        const int at = cols.at(qnorm(c - sv, mod), li);
        if (at >= 0)
          put_range(tp, cols.second.data() + cols.start[at],
                    cols.second.data() + cols.start[at + 1]);
      }
      gs.push_back(g);
    }
  }
  return finish_launch(tp, gs, false, true, S.tile);
}

Launch plan_proj_y(const StepLegs &S, int a0, int a1, const QSet &sA, const QSet &sB,
                   TablePlan &tp) {
  // every output block must take its whole reduction from one group: with
  // several charges on both operands a block (rho, nu) would sum over
  // several kappa (the caller splits such a product by the charge of A)
  if (sA.size() > 1 && sB.size() > 1)
    fail(GXY_EUNSUPPORTED, "projection product with several charges on both operands");
  const int Dh = S.Dh, Dv = S.Dv, mod = S.mod;
  const int64_t W = (int64_t)Dh * Dv;
  // rho = q_a - q_r1 - q_u per row (a, r1, u); kappa = q_l2 - q_i per reduction
  // index (l2, i); nu = q_r2 - q_d per column (r2, d). Each (a, r1) sends the
  // u of one label to one rho, so the rows of a rho stay in (a, r1, u) order.
  const LegLabels V = leg_labels(S.lv, mod);
  const int nl = (int)V.q.size();
  int lo = 0, hi = -1;
  for (int a = a0; a < a1; ++a)
    for (int r1 = 0; r1 < Dh; ++r1)
      for (int li = 0; li < nl; ++li) {
        const int k = qnorm(S.ln[a] - S.lh[r1] - V.q[li], mod);
        if (hi < lo) lo = hi = k;
        lo = std::min(lo, k);
        hi = std::max(hi, k);
      }
  FlatLists rows_by_rho(lo, hi, 1);
  for (int a = a0; a < a1; ++a)
    for (int r1 = 0; r1 < Dh; ++r1)
      for (int li = 0; li < nl; ++li)
        rows_by_rho.start[rows_by_rho.at(qnorm(S.ln[a] - S.lh[r1] - V.q[li], mod), 0) + 1] +=
            (int64_t)V.members[li].size();
  std::vector<int64_t> cur = rows_by_rho.finish_counts();
  for (int a = a0; a < a1; ++a)
    for (int r1 = 0; r1 < Dh; ++r1)
      for (int li = 0; li < nl; ++li) {
        int64_t &c = cur[rows_by_rho.at(qnorm(S.ln[a] - S.lh[r1] - V.q[li], mod), 0)];
        for (int u : V.members[li])
          rows_by_rho.first[c++] = (((int64_t)(a - a0) * Dh + r1) * Dv + u) * W;
      }
  // (l2, i) and (r2, d) in block order: each kappa (nu) is one contiguous range
  std::map<int, std::vector<int64_t>> ks_by_kappa, cols_by_nu;
  for (int l2 = 0; l2 < Dh; ++l2)
    for (int i = 0; i < Dv; ++i)
      ks_by_kappa[qnorm(S.lh[l2] - S.lv[i], mod)].push_back(S.pos[(size_t)l2 * Dv + i]);
  for (int r2 = 0; r2 < Dh; ++r2)
    for (int d = 0; d < Dv; ++d)
      cols_by_nu[qnorm(S.lh[r2] - S.lv[d], mod)].push_back(S.pos[(size_t)r2 * Dv + d]);
  std::vector<int> kappas;
  for (int k = 0; k < rows_by_rho.nk; ++k)
    if (rows_by_rho.size(k) > 0)
      for (int s : sA) kappas.push_back(qnorm(lo + k - s, mod));
  std::sort(kappas.begin(), kappas.end());
  kappas.erase(std::unique(kappas.begin(), kappas.end()), kappas.end());
  // first position and length of a block-order range that must be contiguous
  auto range_of = [](const std::vector<int64_t> &v, int64_t &first) {
    first = v.empty() ? 0 : v.front();
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i] != first + (int64_t)i) fail(GXY_EDEVICE, "block order range is not contiguous");
    return (int32_t)v.size();
  };
  // One group per (kappa, nu): rows through the table, the reduction range
  // of kappa and the column range of nu as bases (contiguous groups). The
  // rows of a kappa enter the table once, before its first group.
  std::vector<GSpec> gs;
  for (int kappa : kappas) {
    int64_t nrows = 0;
    for (int k = 0; k < rows_by_rho.nk; ++k)
      if (rows_by_rho.size(k) > 0 && in_set(qnorm(lo + k - kappa, mod), sA))
        nrows += rows_by_rho.size(k);
    if (nrows == 0) continue;
    int64_t k0 = 0;
    int32_t K = 0;
    auto ik = ks_by_kappa.find(kappa);
    if (ik != ks_by_kappa.end()) K = range_of(ik->second, k0);
    int64_t rows_at = -1;
    for (const auto &kv : cols_by_nu) {
      if (!in_set(qnorm(kappa - kv.first, mod), sB)) continue;
      int64_t c0 = 0;
      const int32_t N = range_of(kv.second, c0);
      if (N == 0) continue;
      if (rows_at < 0) {
        rows_at = (int64_t)tp.tab.size();
        for (int k = 0; k < rows_by_rho.nk; ++k)
          if (rows_by_rho.size(k) > 0 && in_set(qnorm(lo + k - kappa, mod), sA))
            put_range(tp, rows_by_rho.first.data() + rows_by_rho.start[k],
                      rows_by_rho.first.data() + rows_by_rho.start[k + 1]);
      }
      GSpec g;
      g.M = (int32_t)nrows;
      g.N = N;
      g.K = K;
      g.ar = rows_at;
      g.cr = rows_at;
      g.ac = k0;
      g.br = k0 * W + c0;
      g.bc = W;
      g.cc = c0;
      gs.push_back(g);
    }
  }
  return finish_launch(tp, gs, true, true, S.tile, true);
}

Launch plan_proj_t(const StepLegs &S, int a0, int a1, const QSet &sY, TablePlan &tp) {
  const int Dh = S.Dh, Dv = S.Dv, Dn = S.Dn, mod = S.mod;
  const int64_t W = (int64_t)Dh * Dv, per_a = W * W;
  const auto bs = leg_buckets(S.ln, mod);
  const PairBuckets ks = pair_buckets(S.lh, S.lh, 1, 1, mod);  // q_r1 + q_r2
  // rows (a, u, d) keyed by (w = q_a - q_u + q_d, label of d); group
  // (sigma, label) takes the rows with w - sigma in sY. With the label of d
  // fixed, Y's offset splits into a reduction part (r1, pos of (r2, first d
  // of the label)) and a row part (a, u, rank of d in its label).
  const LegLabels V = leg_labels(S.lv, mod);
  const int nl = (int)V.q.size();
  int lo = 0, hi = -1;
  for (int a = a0; a < a1; ++a)
    for (int u = 0; u < Dv; ++u)
      for (int li = 0; li < nl; ++li) {
        const int k = qnorm(S.ln[a] - S.lv[u] + V.q[li], mod);
        if (hi < lo) lo = hi = k;
        lo = std::min(lo, k);
        hi = std::max(hi, k);
      }
  FlatLists rows(lo, hi, nl);
  for (int a = a0; a < a1; ++a)
    for (int u = 0; u < Dv; ++u)
      for (int li = 0; li < nl; ++li)
        rows.start[rows.at(qnorm(S.ln[a] - S.lv[u] + V.q[li], mod), li) + 1] +=
            (int64_t)V.members[li].size();
  std::vector<int64_t> cur = rows.finish_counts();
  for (int a = a0; a < a1; ++a)
    for (int u = 0; u < Dv; ++u)
      for (int li = 0; li < nl; ++li) {
        int64_t &c = cur[rows.at(qnorm(S.ln[a] - S.lv[u] + V.q[li], mod), li)];
        for (int d : V.members[li]) {
          rows.first[c] = (int64_t)(a - a0) * per_a + (int64_t)u * W + S.vrank[d];
          rows.second[c] = (int64_t)a * Dn * Dv * Dv + (int64_t)u * Dv + d;
          ++c;
        }
      }
  // table size of the groups below, so the table grows once
  int64_t total = 0;
  for (const auto &kv : bs) {
    const int sigma = kv.first;
    auto ik = ks.find(sigma);
    const int64_t nk = ik != ks.end() ? (int64_t)ik->second.size() : 0;
    for (int li = 0; li < nl; ++li) {
      int64_t nr = 0;
      for (int sv : sY) nr += rows.size(rows.at(qnorm(sigma + sv, mod), li));
      if (nr) total += 2 * nr + 2 * nk + 2 * (int64_t)kv.second.size();
    }
  }
  tp.tab.reserve(tp.tab.size() + total);
  std::vector<GSpec> gs;
  for (const auto &kv : bs) {
    const int sigma = kv.first;
    std::vector<int64_t> br, bc, cc;
    auto ik = ks.find(sigma);
    if (ik != ks.end())
      for (const PI &p : ik->second) br.push_back(((int64_t)p.first * Dh + p.second) * Dn);
    for (int b : kv.second) {
      bc.push_back(b);
      cc.push_back((int64_t)b * Dv * Dv);
    }
    for (int li = 0; li < nl; ++li) {
      const int d0 = V.members[li][0];
      int64_t nr = 0;
      for (int sv : sY) nr += rows.size(rows.at(qnorm(sigma + sv, mod), li));
      if (nr == 0) continue;
      GSpec g;
      g.M = (int32_t)nr;
      g.N = (int32_t)bc.size();
      g.K = ik != ks.end() ? (int32_t)ik->second.size() : 0;
      g.ar = (int64_t)tp.tab.size();
      for (int sv : sY) {
        const int at = rows.at(qnorm(sigma + sv, mod), li);
        if (at >= 0)
          put_range(tp, rows.first.data() + rows.start[at], rows.first.data() + rows.start[at + 1]);
      }
      g.ac = (int64_t)tp.tab.size();
      if (ik != ks.end())
        for (const PI &p : ik->second)
          tp.tab.push_back((int64_t)p.first * Dv * W + S.pos[(size_t)p.second * Dv + d0]);
      g.br = put(tp, br);
      g.bc = put(tp, bc);
      g.cr = (int64_t)tp.tab.size();
      for (int sv : sY) {
        const int at = rows.at(qnorm(sigma + sv, mod), li);
        if (at >= 0)
          put_range(tp, rows.second.data() + rows.start[at],
                    rows.second.data() + rows.start[at + 1]);
      }
      g.cc = put(tp, cc);
      gs.push_back(g);
    }
  }
  return finish_launch(tp, gs, false, true, S.tile);
}

}  // namespace gxy
