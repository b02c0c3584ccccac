// Host orchestration of HOTRG runs and the C ABI (include/gxy_hotrg.h).
//
// One run (Ch. 2 HOTRG on the Ch. 3 gXY site tensor):
//   t_n, field factors, T and impurity tensors      (device, FP64)
//   normalise (Frobenius), log-norm accumulation   (device, FP64)
//   for each step: [transpose for x-steps]
//     environments E_L, E_R of the fused two-site tensor (FP64 MFMA GEMMs)
//     per-sector block-Jacobi eigensolve (FP64), truncation with the tie
//     rule and side choice (device), projector P
//     T' = P^T M P in three GEMMs chunked over the output index, impurity
//     tensors symmetrised, normalise          [transpose back]
//   trace, ln Z / V and <cos theta>, <cos 2 theta> (device)
// The host only plans launches: it reads back the symmetry labels of the
// kept states after each truncation to size the next step's sectors.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <future>
#include <mutex>
#include <thread>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/gxy_hotrg_testing.h"
#include "ctx.h"
#include "internal.h"
#include "plan.h"

namespace gxy {

constexpr double kTieRel = 1e-12;
constexpr double kSideTol = 1e-10;
constexpr int kMaxSweeps = 120;
constexpr size_t kPlanAhead = 16;                // projection launches planned ahead
// projection chunk bound over the three D^5 buffers (X, X of an impurity, Y):
// 32 GiB keeps Dcut = 64 with both impurity chains in one chunk
constexpr size_t kDefaultChunkBytes = (size_t)32 << 30;
constexpr int kLmax = 50;

enum Sym { SYM_U1 = 0, SYM_NONE = 1, SYM_Z2 = 2 };

static bool env_flag(const char *name) {
  const char *v = getenv(name);
  return v && *v && strcmp(v, "0") != 0;
}

static size_t env_size(const char *name, size_t dflt) {
  const char *v = getenv(name);
  if (!v || !*v) return dflt;
  return (size_t)strtoull(v, nullptr, 10);
}

// ---------------------------------------------------------------------------
// workspace: one device block carved into aligned pieces
// ---------------------------------------------------------------------------

struct Carver {
  size_t off = 0;
  char *base = nullptr;
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct StepDims {
  int dh, dv, dn;  // in y-orientation: legs l/r = dh, u/d = dv; output dn
  bool xstep;
};

struct Plan {
  int d0;
  std::vector<StepDims> steps;
  int64_t maxT = 0;       // elements of the largest site tensor
  int64_t maxNF = 0;      // largest fused dimension that gets truncated
  int64_t maxNFall = 0;   // largest fused dimension
  int64_t maxPD = 0;      // largest P (nf * dn)
  int maxDn = 0;
  int64_t chunk_elems = 0;  // X / Y chunk buffer elements
  int64_t maxW = 0;         // largest fused (horizontal, vertical) dimension
  int nimp = 0;
  int64_t tab_env = 0, tab_proj = 0;  // offset-table entries (bounds)
  int64_t grp_env = 0, grp_proj = 0;  // group descriptors (bounds)
  int64_t proj_bytes = 0;             // projection slices of one step (bound)
  // impurity projections on a second stream, one step behind the pure
  // tensor's chain (charge blocks, impurities, one chunk per step)
  bool overlap = false;
};

static int sym_of(const gxy_point &p);

// Impurity chains of a run: the one-insertion chains (cos theta, cos q theta)
// first, then the second-moment chains, each with the index of the
// one-insertion chain it is built from. A second moment carries its first
// moment along.
struct Chains {
  int n = 0;
  int which[4] = {0, 0, 0, 0};   // GXY_IMP_* of chain k
  int first[4] = {-1, -1, -1, -1};  // second-moment chains: their first moment
};

static Chains chains_of(const gxy_point &p) {
  Chains c;
  uint32_t m = p.impurities;
  if (m & GXY_IMP_COS1_SQ) m |= GXY_IMP_COS1;
  if (m & GXY_IMP_COS2_SQ) m |= GXY_IMP_COS2;
  int at1 = -1, at2 = -1;
  if (m & GXY_IMP_COS1) { at1 = c.n; c.which[c.n++] = GXY_IMP_COS1; }
  if (m & GXY_IMP_COS2) { at2 = c.n; c.which[c.n++] = GXY_IMP_COS2; }
  if (m & GXY_IMP_COS1_SQ) { c.first[c.n] = at1; c.which[c.n++] = GXY_IMP_COS1_SQ; }
  if (m & GXY_IMP_COS2_SQ) { c.first[c.n] = at2; c.which[c.n++] = GXY_IMP_COS2_SQ; }
  return c;
}

static Plan make_plan(const gxy_point &p, size_t chunk_bytes, bool allow_overlap = true) {
  Plan pl;
  pl.d0 = 2 * p.nmax + 1;
  int Dh = pl.d0, Dv = pl.d0;
  pl.nimp = chains_of(p).n;
  pl.maxT = (int64_t)Dh * Dh * Dv * Dv;
  int64_t per_a_max = 1;
  for (int n = 1; n <= p.nsteps; ++n) {
    const bool xs = (n % 2 == 0);
    StepDims sd;
    sd.xstep = xs;
    sd.dh = xs ? Dv : Dh;
    sd.dv = xs ? Dh : Dv;
    const int64_t nf = (int64_t)sd.dh * sd.dh;
    sd.dn = (int)std::min<int64_t>(p.dcut, nf);
    pl.steps.push_back(sd);
    const int64_t t_in = (int64_t)sd.dh * sd.dh * sd.dv * sd.dv;
    const int64_t t_out = (int64_t)sd.dn * sd.dn * sd.dv * sd.dv;
    pl.maxT = std::max({pl.maxT, t_in, t_out});
    pl.maxNFall = std::max(pl.maxNFall, nf);
    if (nf > p.dcut) pl.maxNF = std::max(pl.maxNF, nf);
    pl.maxPD = std::max(pl.maxPD, nf * sd.dn);
    pl.maxDn = std::max(pl.maxDn, sd.dn);
    per_a_max = std::max(per_a_max, (int64_t)sd.dh * sd.dv * sd.dh * sd.dv);
    pl.maxW = std::max(pl.maxW, (int64_t)sd.dh * sd.dv);
    if (xs)
      Dv = sd.dn;
    else
      Dh = sd.dn;
  }
  // chunk buffers: X (pure), X (impurity) and Y, each ac * per_a elements
  const int nbuf = pl.nimp > 0 ? 3 : 2;
  int64_t ac = (int64_t)(chunk_bytes / (sizeof(double) * nbuf * per_a_max));
  ac = std::max<int64_t>(1, std::min<int64_t>(ac, pl.maxDn));
  pl.chunk_elems = ac * per_a_max;
  pl.overlap = allow_overlap && sym_of(p) != SYM_NONE && pl.nimp > 0 && ac >= pl.maxDn &&
               !getenv("GXY_NO_OVERLAP");
  // Bounds of the charge-block tables of one step (see plan.hip), per launch
  // with s the number of charges of its charged factor (a column of X, a row
  // of Y or T' appears in at most s groups; a label slot repeats the row and
  // reduction lists at most Dv times): X 2 ac Dh Dv + 2 Dh Dv + 2 s Dh Dv^2,
  // Y (rows only) s ac Dh Dv, T' 2 Dh^2 Dv + 2 Dn Dv + 2 s ac Dv^2.
  // Launches per chunk: pure X, Y, T'; a one-insertion chain (charges s1)
  // Y(1) X(s1) Y(s1) T'(s1); a second-moment chain (charges 3, first moment
  // 2) Y(1) X(3) Y(3) X(2) Y(1) Y(1) T'(3).
  const Chains chn = chains_of(p);
  const int64_t nvar = 1 + 3 * pl.nimp;
  for (const StepDims &sd : pl.steps) {
    const int64_t Dh = sd.dh, Dv = sd.dv, Dn = sd.dn, MN = Dh * Dv;
    const int64_t nch = (Dn + ac - 1) / ac;
    const int64_t env = 2 * (8 * MN + 4 * Dh * Dh + Dv * Dv) + 64;
    const int64_t acn = std::min<int64_t>(ac, Dn);
    auto bx = [&](int64_t sc) { return 2 * acn * Dh * Dv + 2 * Dh * Dv + 2 * sc * Dh * Dv * Dv + 64; };
    auto by = [&](int64_t sc) { return sc * acn * Dh * Dv + 64; };
    auto bt = [&](int64_t sc) { return 2 * Dh * Dh * Dv + 2 * Dn * Dv + 2 * sc * acn * Dv * Dv + 64; };
    int64_t per_chunk = bx(1) + by(1) + bt(1);
    for (int k = 0; k < chn.n; ++k)
      per_chunk += chn.first[k] < 0 ? by(1) + bx(2) + by(2) + bt(2)
                                    : by(1) + bx(3) + by(3) + bx(2) + 2 * by(1) + bt(3);
    const int64_t proj = nch * per_chunk + 64;
    pl.tab_env = std::max(pl.tab_env, env);
    pl.tab_proj = std::max(pl.tab_proj, proj);
    pl.grp_env = std::max(pl.grp_env, 2 * (2 * MN + Dh * Dh) + 16);
    pl.grp_proj = std::max(pl.grp_proj, nch * nvar * (Dn * Dh + 2 * MN + Dn + 16));
    // one slice per launch (groups, then tables), each rounded up to 64 bytes
    const int64_t nlaunch = nch * (3 + 6 * pl.nimp);
    pl.proj_bytes = std::max(pl.proj_bytes, 8 * pl.tab_proj +
                                                (int64_t)sizeof(GGroup) * pl.grp_proj +
                                                64 * nlaunch);
  }
  return pl;
}

struct Buffers {
  double *T, *Tn, *T2;             // site tensor, next, bottom-operand copy
  double *TX[4], *TXn[4], *TX2[4]; // impurity tensors
  double *envA, *envB, *E;         // environments
  double *P;                       // projector of the current step
  double *X, *XI, *Y, *YI;         // projection chunks (YI: impurity stream)
  // per step parity: what the impurity stream of step n reads while the
  // pure chain runs step n + 1
  double *Pb[2], *Xb[2], *T2b[2];
  int32_t *permb[2];
  char *tabb[2];
  double *eigA, *eigV, *eigQ, *eigB1, *eigB2;
  int64_t *gtab;
  GGroup *ggrp;
  int64_t gtab_cap, ggrp_cap;
  double *eig_scale;
  int32_t *eig_flags;
  int32_t *ints;                   // sector / pair / tile tables
  int64_t ints_cap;
  double *sel_lam;
  int32_t *sel_int;                // cand sec, rank, col, taken + side picks
  int32_t *pick;                   // pick sec, col, label
  double *diag;                    // 24
  double *partial;                 // norm partials
  double *nrm;                     // 3 * (nsteps + 1)
  double *coef;                    // t, F, FM, FM1
  double *scal;                    // traces and result
  int64_t *tab_env;                // charge-block offset tables
  char *proj_tab;                  // projection slices: groups + tables
  int32_t *perm;                   // inverse block order of the fused index
  GGroup *grp_env;
  int64_t eig_elems, eig_q;
  int64_t sel_cap;
};

static size_t carve(const gxy_point &p, const Plan &pl, Carver &c, Buffers &b) {
  const int64_t T = pl.maxT;
  b.T = c.take<double>(T);
  b.Tn = c.take<double>(T);
  b.T2b[0] = c.take<double>(T);
  b.T2b[1] = pl.overlap ? c.take<double>(T) : b.T2b[0];
  b.T2 = b.T2b[0];
  for (int k = 0; k < 4; ++k) {
    const bool on = k < pl.nimp;
    b.TX[k] = on ? c.take<double>(T) : nullptr;
    b.TXn[k] = on ? c.take<double>(T) : nullptr;
    b.TX2[k] = on ? c.take<double>(T) : nullptr;
  }
  b.envA = c.take<double>(T);
  b.envB = c.take<double>(T);
  const int64_t nf = pl.maxNF;
  b.E = c.take<double>(2 * nf * nf);
  b.Pb[0] = c.take<double>(std::max<int64_t>(pl.maxPD, 1));
  b.Pb[1] = pl.overlap ? c.take<double>(std::max<int64_t>(pl.maxPD, 1)) : b.Pb[0];
  b.P = b.Pb[0];
  b.Xb[0] = c.take<double>(pl.chunk_elems);
  b.Xb[1] = pl.overlap ? c.take<double>(pl.chunk_elems) : b.Xb[0];
  b.X = b.Xb[0];
  b.XI = pl.nimp > 0 ? c.take<double>(pl.chunk_elems) : nullptr;
  b.Y = c.take<double>(pl.chunk_elems);
  b.YI = pl.overlap ? c.take<double>(pl.chunk_elems) : b.Y;
  // eigen: per side sum of npad^2 <= nf^2 + 1023 nf
  b.eig_elems = 2 * (nf * nf + 1023 * nf);
  b.eigA = c.take<double>(std::max<int64_t>(b.eig_elems, 1));
  b.eigV = c.take<double>(std::max<int64_t>(b.eig_elems, 1));
  b.eigB1 = c.take<double>(std::max<int64_t>(b.eig_elems, 1));
  b.eigB2 = c.take<double>(std::max<int64_t>(b.eig_elems, 1));
  // batched-product tables: 4 entries per padded row, 2 groups per matrix
  b.gtab_cap = 256 * nf + 64;
  b.ggrp_cap = 2 * 2 * nf + 8;
  b.gtab = c.take<int64_t>(b.gtab_cap);
  b.ggrp = c.take<GGroup>(b.ggrp_cap);
  b.eig_q = 2 * nf * 1024 + 1024;
  b.eigQ = c.take<double>(b.eig_q);
  b.eig_scale = c.take<double>(2 * nf + 2);
  b.eig_flags = c.take<int32_t>(4 * nf + 4 + 2 * nf + 4);  // flags, next flags, pair_rot
  // tables: sec idx (nf), start/n/label (3 nf), mats (2*2nf npad + 2*2nf off
  // as 2 ints), pairbase (2nf+1), pair_mat (<= 2 nf), tiles (4 * bound)
  const int64_t nmat = 2 * nf;
  const int64_t pairs = 2 * nf;
  // update tiles per matrix: q(q-1)/2 + q^2 with q = ceil(n/32); summed over
  // both sides q^2 <= (n/32 + 1)^2 gives <= 1.5 (2 nf^2/1024 + nf/8 + 2 nf)
  const int64_t tiles = (3 * (2 * nf * nf / 1024 + nf / 8 + 2 * nf)) / 2 + 16;
  b.ints_cap = nf + 3 * nf + nmat + 2 * nmat + (nmat + 1) + pairs + 4 * tiles + 64;
  b.ints = c.take<int32_t>(b.ints_cap);
  b.sel_cap = 2 * nf;
  b.sel_lam = c.take<double>(2 * nf + 2);
  b.sel_int = c.take<int32_t>(4 * 2 * nf + 6 * (int64_t)std::max(pl.maxDn, 1) + 8);
  b.pick = c.take<int32_t>(3 * (int64_t)std::max(pl.maxDn, 1) + 8);
  b.diag = c.take<double>(32);
  b.partial = c.take<double>(1024);
  b.nrm = c.take<double>(3 * (int64_t)(p.nsteps + 1));
  const int qmax = 4 * p.nmax;
  b.coef = c.take<double>(pl.d0 + 5 * (2 * qmax + 1));
  b.scal = c.take<double>(16);
  b.tab_env = c.take<int64_t>(pl.tab_env);
  for (int q = 0; q < 2; ++q) {
    b.permb[q] = (q == 0 || pl.overlap) ? c.take<int32_t>(std::max<int64_t>(pl.maxW, 1))
                                        : b.permb[0];
    b.tabb[q] = (q == 0 || pl.overlap) ? c.take<char>(pl.proj_bytes) : b.tabb[0];
  }
  b.perm = b.permb[0];
  b.proj_tab = b.tabb[0];
  b.grp_env = c.take<GGroup>(pl.grp_env);
  return c.off + 256;
}

}  // namespace gxy

namespace gxy {

// One stream per run and no cooperative launches: batch workers (many of
// them already fill the device) and no-allocation runs.
static bool single_stream(const gxy_ctx *ctx) { return ctx->worker || ctx->noalloc; }

static void ensure_pinned(gxy_ctx *ctx, size_t bytes) {
  if (ctx->noalloc) return;   // host staging is ctx->noalloc_host
  if (ctx->pinned_bytes >= bytes) return;
  if (ctx->pinned) GXY_HIP(hipHostFree(ctx->pinned));
  ctx->pinned = nullptr;
  ctx->pinned_bytes = 0;
  GXY_HIP(hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault));
  ctx->pinned_bytes = bytes;
}

// Copy a table plan to the device through pinned staging buffer j; the
// buffer is reused only after its previous copy has completed.
static void upload_plan(gxy_ctx *ctx, int j, const TablePlan &tp, int64_t *d_tab,
                        int64_t tab_cap, GGroup *d_grp, int64_t grp_cap, hipStream_t s) {
  if ((int64_t)tp.tab.size() > tab_cap || (int64_t)tp.groups.size() > grp_cap)
    fail(GXY_ENOMEM, "charge-block table bound exceeded");
  const size_t tb = tp.tab.size() * sizeof(int64_t), gb = tp.groups.size() * sizeof(GGroup);
  if (ctx->noalloc) {
    // straight from the planner's host vectors, complete before they go
    if (tb) GXY_HIP(hipMemcpyAsync(d_tab, tp.tab.data(), tb, hipMemcpyHostToDevice, s));
    if (gb) GXY_HIP(hipMemcpyAsync(d_grp, tp.groups.data(), gb, hipMemcpyHostToDevice, s));
    GXY_HIP(hipStreamSynchronize(s));
    return;
  }
  const size_t need = tb + gb + 64;
  if (ctx->stage_used[j]) GXY_HIP(hipEventSynchronize(ctx->stage_ev[j]));
  if (ctx->stage_bytes[j] < need) {
    if (ctx->stage[j]) GXY_HIP(hipHostFree(ctx->stage[j]));
    ctx->stage[j] = nullptr;
    GXY_HIP(hipHostMalloc(&ctx->stage[j], need + need / 2, hipHostMallocDefault));
    ctx->stage_bytes[j] = need + need / 2;
  }
  if (!ctx->stage_ev[j]) GXY_HIP(hipEventCreateWithFlags(&ctx->stage_ev[j], hipEventDisableTiming));
  char *h = (char *)ctx->stage[j];
  memcpy(h, tp.tab.data(), tb);
  memcpy(h + tb, tp.groups.data(), gb);
  if (tb) GXY_HIP(hipMemcpyAsync(d_tab, h, tb, hipMemcpyHostToDevice, s));
  if (gb) GXY_HIP(hipMemcpyAsync(d_grp, h + tb, gb, hipMemcpyHostToDevice, s));
  GXY_HIP(hipEventRecord(ctx->stage_ev[j], s));
  ctx->stage_used[j] = true;
}

// Projection tables of one step: every launch is planned on a host thread
// and copied into its own slice of a pinned arena (its group descriptors,
// then its offset tables); slices are taken by an atomic bump and the
// device area mirrors the arena, so a slice's device copy is one contiguous
// copy at the same offset. The copies run on a side stream and the compute
// stream waits for each before its launch. The arena is reused once the
// previous step's copies have completed.
struct ProjArena {
  char *base = nullptr;
  int64_t cap = 0;
  std::atomic<int64_t> used{0};
  int32_t *perm = nullptr;  // block-order permutation of the step
};

static void proj_stage_begin(gxy_ctx *ctx, int q, ProjArena &A, int64_t cap, int64_t perm_cap,
                             hipStream_t s) {
  if (ctx->noalloc) {
    // one host arena (host heap), reused once the stream has drained
    GXY_HIP(hipStreamSynchronize(s));
    const size_t cb = ((size_t)cap + 255) & ~(size_t)255;
    const size_t need = cb + (size_t)perm_cap * sizeof(int32_t) + 256;
    if (ctx->noalloc_arena.size() < need) ctx->noalloc_arena.resize(need);
    char *b = ctx->noalloc_arena.data();
    b += (256 - ((uintptr_t)b & 255)) & 255;
    A.base = b;
    A.cap = cap;
    A.used = 0;
    A.perm = (int32_t *)(A.base + cb);
    return;
  }
  if (ctx->arena_pending[q]) GXY_HIP(hipEventSynchronize(ctx->arena_ev[q]));
  ctx->arena_pending[q] = false;
  const size_t cb = ((size_t)cap + 255) & ~(size_t)255;
  const size_t need = cb + (size_t)perm_cap * sizeof(int32_t);
  if (ctx->arena_bytes[q] < need) {
    if (ctx->arena[q] && !ctx->arena_pageable[q]) GXY_HIP(hipHostFree(ctx->arena[q]));
    ctx->arena[q] = nullptr;
    ctx->arena_bytes[q] = 0;
    ctx->arena_pageable[q] = false;
    if (hipHostMalloc(&ctx->arena[q], need, hipHostMallocDefault) != hipSuccess) {
      // pinned memory exhausted (many worker contexts): pageable host
      // memory, whose copies the runtime completes before returning
      (void)hipGetLastError();
      ctx->arena_host[q].resize(need + 256);
      char *b = ctx->arena_host[q].data();
      ctx->arena[q] = b + ((256 - ((uintptr_t)b & 255)) & 255);
      ctx->arena_pageable[q] = true;
    }
    ctx->arena_bytes[q] = need;
  }
  A.base = (char *)ctx->arena[q];
  A.cap = cap;
  A.used = 0;
  A.perm = (int32_t *)(A.base + cb);
}

// After the last launch of a step that reads arena q's tables (on stream s):
// the arena may be reused once this event has completed (every copy
// precedes its launch).
static void proj_stage_done(gxy_ctx *ctx, int q, hipStream_t s) {
  if (ctx->noalloc) return;   // the next step's begin drains the stream
  if (!ctx->arena_ev[q])
    GXY_HIP(hipEventCreateWithFlags(&ctx->arena_ev[q], hipEventDisableTiming));
  GXY_HIP(hipEventRecord(ctx->arena_ev[q], s));
  ctx->arena_pending[q] = true;
}

// Stream b waits for what stream a has been given so far (no-op for a == b).
static void stream_after(gxy_ctx *ctx, hipStream_t b, hipStream_t a, int slot) {
  if (a == b) return;
  if (!ctx->pipe_ev[slot]) GXY_HIP(hipEventCreateWithFlags(&ctx->pipe_ev[slot], hipEventDisableTiming));
  GXY_HIP(hipEventRecord(ctx->pipe_ev[slot], a));
  GXY_HIP(hipStreamWaitEvent(b, ctx->pipe_ev[slot], 0));
}

// One planned projection launch and its slice of the arena.
struct ProjJob {
  Launch L;
  int64_t off = 0, bytes = 0, ngrp = 0;
  bool sent = false;
};

// Host-thread side: copy a finished plan into a fresh slice of the arena.
static void stage_plan(ProjArena &A, const TablePlan &tp, const Launch &L, ProjJob &j) {
  j.L = L;
  j.ngrp = (int64_t)tp.groups.size();
  const int64_t gb = j.ngrp * (int64_t)sizeof(GGroup);
  const int64_t tb = (int64_t)tp.tab.size() * (int64_t)sizeof(int64_t);
  j.bytes = (gb + tb + 63) & ~(int64_t)63;
  j.off = A.used.fetch_add(j.bytes);
  if (j.off + j.bytes > A.cap) fail(GXY_ENOMEM, "charge-block table bound exceeded");
  if (gb) memcpy(A.base + j.off, tp.groups.data(), gb);
  if (tb) memcpy(A.base + j.off + gb, tp.tab.data(), tb);
}

// Stream side: the slice's device copy (once per job) on the side stream,
// ordered before the compute stream's next launch.
static void send_plan(gxy_ctx *ctx, const ProjArena &A, ProjJob &j, char *d_area, hipStream_t s,
                      size_t k) {
  if (j.sent) return;
  if (j.bytes && single_stream(ctx)) {   // copy on the run's own stream
    GXY_HIP(hipMemcpyAsync(d_area + j.off, A.base + j.off, j.bytes, hipMemcpyHostToDevice, s));
  } else if (j.bytes) {
    while (ctx->copy_ev.size() <= k) {
      hipEvent_t e;
      GXY_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ctx->copy_ev.push_back(e);
    }
    GXY_HIP(hipMemcpyAsync(d_area + j.off, A.base + j.off, j.bytes, hipMemcpyHostToDevice,
                           ctx->copy_stream));
    GXY_HIP(hipEventRecord(ctx->copy_ev[k], ctx->copy_stream));
    GXY_HIP(hipStreamWaitEvent(s, ctx->copy_ev[k], 0));
  }
  j.sent = true;
}

static void run_launch(const Launch &L, const GGroup *d_grp, const int64_t *d_tab,
                       const double *A, const double *B, double *C, double alpha, double beta,
                       hipStream_t s, int prec = GXY_PREC_FP64, bool dma = false) {
  GroupedGemm g{};
  g.dma = dma;
  g.sym = L.sym;
  if (L.sym && beta != 0.0) fail(GXY_EDEVICE, "symmetric launch with beta != 0");
  g.prec = prec;
  g.ngroups = L.ngroups;
  g.total_tiles = L.total_tiles;
  g.tile = L.tile;
  g.groups = d_grp + L.first_group;
  g.tab = d_tab;
  g.A = A;
  g.B = B;
  g.C = C;
  g.alpha = alpha;
  g.beta = beta;
  g.kfast_a = L.kfast_a;
  g.nfast_b = L.nfast_b;
  g.contig = L.contig;
  grouped_gemm(g, s);
}

static void ensure_workspace(gxy_ctx *ctx, size_t need) {
  if (ctx->ws && ctx->ws_bytes >= need) return;
  if (ctx->noalloc)
    fail(GXY_EINVAL, "the run needs " + std::to_string(need) +
                         " bytes of device workspace; the no-allocation scratch holds " +
                         std::to_string(ctx->ws_bytes));
  if (ctx->ws && !ctx->ws_owned)
    fail(GXY_ENOMEM, "caller workspace of " + std::to_string(ctx->ws_bytes) +
                         " bytes is smaller than the " + std::to_string(need) +
                         " bytes needed");
  if (ctx->ws) GXY_HIP(hipFree(ctx->ws));
  ctx->ws = nullptr;
  ctx->ws_bytes = 0;
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(GXY_ENOMEM, "hipMalloc of " + std::to_string(need) + " bytes failed");
  }
  ctx->ws = p;
  ctx->ws_bytes = need;
  ctx->ws_owned = true;
}

// Events around each launch of the hot contraction (enabled by GXY_TIMING).
static void hot_begin(gxy_ctx *ctx, hipStream_t s, double flops, double bytes) {
  if (!ctx->hot_on) return;
  const size_t k = ctx->hot_launches.size();
  while (ctx->ev_pool.size() < 2 * (k + 1)) {
    hipEvent_t e;
    GXY_HIP(hipEventCreate(&e));
    ctx->ev_pool.push_back(e);
  }
  GXY_HIP(hipEventRecord(ctx->ev_pool[2 * k], s));
  ctx->hot_launches.push_back({(int)k, flops});
  ctx->hot_stats[3] += bytes;
}

static void hot_end(gxy_ctx *ctx, hipStream_t s) {
  if (!ctx->hot_on) return;
  const size_t k = ctx->hot_launches.size() - 1;
  GXY_HIP(hipEventRecord(ctx->ev_pool[2 * k + 1], s));
}

static void hot_collect(gxy_ctx *ctx) {
  if (!ctx->hot_on) return;
  for (auto &pr : ctx->hot_launches) {
    float ms = 0;
    GXY_HIP(hipEventSynchronize(ctx->ev_pool[2 * pr.first + 1]));
    GXY_HIP(hipEventElapsedTime(&ms, ctx->ev_pool[2 * pr.first], ctx->ev_pool[2 * pr.first + 1]));
    ctx->hot_stats[0] += 1;
    ctx->hot_stats[1] += ms;
    ctx->hot_stats[2] += pr.second;
  }
  ctx->hot_launches.clear();
}

static void validate(const gxy_point &p) {
  if (!(p.beta >= 0.0) || !isfinite(p.beta)) fail(GXY_EINVAL, "beta must be finite and >= 0");
  if (!(p.delta >= 0.0 && p.delta <= 1.0)) fail(GXY_EINVAL, "delta must lie in [0, 1]");
  if (!isfinite(p.h) || !isfinite(p.h1)) fail(GXY_EINVAL, "fields must be finite");
  if (p.nmax < 0 || p.nmax > 64) fail(GXY_EINVAL, "nmax must lie in [0, 64]");
  if (p.dcut < 1 || p.dcut > 128) fail(GXY_EINVAL, "dcut must lie in [1, 128]");
  if (p.nsteps < 0 || p.nsteps > 62) fail(GXY_EINVAL, "nsteps must lie in [0, 62]");
  if (p.nquad <= 2 * p.nmax) fail(GXY_EINVAL, "nquad must exceed 2*nmax");
  if (p.impurities & ~15u) fail(GXY_EINVAL, "unknown impurity bits");
  if ((p.impurities & (GXY_IMP_COS1_SQ | GXY_IMP_COS2_SQ)) && (p.h != 0.0 || p.h1 != 0.0))
    fail(GXY_EUNSUPPORTED, "second-moment insertions are built at zero field only");
  if (p.prec != GXY_PREC_FP64 && p.prec != GXY_PREC_FP32 && p.prec != GXY_PREC_BF16X3)
    fail(GXY_EINVAL, "unknown contraction precision");
  if (p.fp64_steps < 0) fail(GXY_EINVAL, "fp64_steps must be >= 0");
  if (p.q != 0 && (p.q < 2 || p.q > 16)) fail(GXY_EINVAL, "q must be 0 (= 2) or lie in [2, 16]");
}

// harmonic of the second coupling (0 selects the thesis's q = 2)
static int harmonic(const gxy_point &p) { return p.q == 0 ? 2 : p.q; }

static int sym_of(const gxy_point &p) {
  if (p.h == 0.0 && p.h1 == 0.0) return SYM_U1;
  if (p.h == 0.0) return SYM_Z2;
  return SYM_NONE;
}

// labels fuse by addition (U(1)), by addition mod q (Z_q), or not at all
static int fuse(int a, int b, int sym, int q) {
  if (sym == SYM_U1) return a + b;
  if (sym == SYM_Z2) return (((a + b) % q) + q) % q;
  return 0;
}

struct Timer {
  bool on = false;
  hipStream_t s = nullptr;
  double *acc = nullptr;
  hipEvent_t a{}, b{};
  void begin() {
    if (on) GXY_HIP(hipEventRecord(a, s));
  }
  void end(int phase) {
    if (!on) return;
    GXY_HIP(hipEventRecord(b, s));
    GXY_HIP(hipEventSynchronize(b));
    float ms = 0;
    GXY_HIP(hipEventElapsedTime(&ms, a, b));
    acc[phase] += ms;
  }
};

// ---------------------------------------------------------------------------
// GEMM helpers for the contractions of one y-step
// ---------------------------------------------------------------------------

// A_env[(l1,i),(l1',i')] = sum_{r1,u} T[l1,r1,u,i] T[l1',r1,u,i']   (left)
// B_env[(l2,i),(l2',i')] = sum_{r2,d} T[l2,r2,i,d] T[l2',r2,i',d]   (left)
// right side: r and l exchanged.
static void env_gemms(const double *T, int Dh, int Dv, double *envA, double *envB,
                      double *E, bool right, hipStream_t s) {
  const int64_t sl = (int64_t)Dh * Dv * Dv, sr = (int64_t)Dv * Dv;
  const int32_t MN = Dh * Dv;
  GemmDesc g{};
  // Gram over (outer leg, u) for the top tensor: rows (x, i), x = l1 or r1
  g.M = MN;
  g.N = MN;
  g.K = MN;
  g.A = T;
  g.B = T;
  g.C = envA;
  g.alpha = 1.0;
  g.beta = 0.0;
  if (!right) {
    g.am = imap2(Dv, sl, 1);       // (l1, i)
    g.ak = imap2(Dv, sr, Dv);      // (r1, u)
  } else {
    g.am = imap2(Dv, sr, 1);       // (r1, i)
    g.ak = imap2(Dv, sl, Dv);      // (l1, u)
  }
  g.bk = g.ak;
  g.bn = g.am;
  g.cm = imap1(MN);
  g.cn = imap1(1);
  g.kfast_a = false;
  g.nfast_b = true;
  gemm(g, s);
  // bottom tensor: rows (x, i), reduction (other leg, d)
  if (!right) {
    g.am = imap2(Dv, sl, Dv);      // (l2, i)
    g.ak = imap2(Dv, sr, 1);       // (r2, d)
  } else {
    g.am = imap2(Dv, sr, Dv);      // (r2, i)
    g.ak = imap2(Dv, sl, 1);       // (l2, d)
  }
  g.bk = g.ak;
  g.bn = g.am;
  g.C = envB;
  g.kfast_a = true;
  g.nfast_b = false;
  gemm(g, s);
  // E[(x1,x2),(x1',x2')] = sum_{i,i'} envA[x1,i,x1',i'] envB[x2,i,x2',i']
  GemmDesc e{};
  e.M = Dh * Dh;
  e.N = Dh * Dh;
  e.K = Dv * Dv;
  e.A = envA;
  e.B = envB;
  e.C = E;
  e.alpha = 1.0;
  e.beta = 0.0;
  const int64_t row = (int64_t)Dv * Dh * Dv;
  e.am = imap2(Dh, row, Dv);                    // (x1, x1')
  e.ak = imap2(Dv, (int64_t)Dh * Dv, 1);        // (i, i')
  e.bk = e.ak;
  e.bn = imap2(Dh, row, Dv);                    // (x2, x2')
  const int64_t nf = (int64_t)Dh * Dh;
  e.cm = imap2(Dh, nf * Dh, Dh);                // row (x1,x2), col (x1',x2')
  e.cn = imap2(Dh, nf, 1);
  e.kfast_a = true;
  e.nfast_b = false;
  gemm(e, s);
}

// X[a][r1][u][l2][i] = sum_{l1} P[(l1,l2), a0 + a] A[l1][r1][u][i], a < ac
static void proj_x(const double *P, int Dh, int Dv, int Dn, int a0, int ac,
                   const double *A, double *X, hipStream_t s, int prec) {
  GemmDesc g{};
  g.prec = prec;
  g.M = ac * Dh;
  g.N = Dh * Dv * Dv;
  g.K = Dh;
  g.A = P + a0;
  g.am = imap2(Dh, 1, Dn);                        // (a, l2)
  g.ak = imap1((int64_t)Dh * Dn);                 // l1
  g.B = A;
  g.bk = imap1((int64_t)Dh * Dv * Dv);
  g.bn = imap1(1);                                // (r1, u, i)
  g.C = X;
  const int64_t per_a = (int64_t)Dh * Dv * Dh * Dv;
  g.cm = imap2(Dh, per_a, Dv);                    // (a, l2)
  g.cn = imap3(Dv, Dv, (int64_t)Dv * Dh * Dv, (int64_t)Dh * Dv, 1);  // (r1, u, i)
  g.alpha = 1.0;
  g.beta = 0.0;
  g.kfast_a = false;
  g.nfast_b = true;
  gemm(g, s);
}

// Y[(a,r1,u),(r2,d)] = sum_{(l2,i)} X[(a,r1,u),(l2,i)] B2[(l2,i),(r2,d)]
static void proj_y(const double *X, const double *B2, int Dh, int Dv, int ac,
                   double *Y, hipStream_t s, int prec) {
  GemmDesc g{};
  g.prec = prec;
  const int32_t W = Dh * Dv;
  g.M = ac * W;
  g.N = W;
  g.K = W;
  g.A = X;
  g.am = imap1(W);
  g.ak = imap1(1);
  g.B = B2;
  g.bk = imap1(W);
  g.bn = imap1(1);
  g.C = Y;
  g.cm = imap1(W);
  g.cn = imap1(1);
  g.alpha = 1.0;
  g.beta = 0.0;
  g.kfast_a = true;
  g.nfast_b = true;
  gemm(g, s);
}

// T'[a0+a][b][u][d] = alpha sum_{r1,r2} Y[a][r1][u][r2][d] P[(r1,r2), b] + beta T'
static void proj_t(const double *Y, const double *P, int Dh, int Dv, int Dn, int a0,
                   int ac, double alpha, double beta, double *Tout, hipStream_t s, int prec) {
  GemmDesc g{};
  g.prec = prec;
  g.M = ac * Dv * Dv;
  g.N = Dn;
  g.K = Dh * Dh;
  g.A = Y;
  const int64_t per_a = (int64_t)Dh * Dv * Dh * Dv;
  g.am = imap3(Dv, Dv, per_a, (int64_t)Dh * Dv, 1);          // (a, u, d)
  g.ak = imap2(Dh, (int64_t)Dv * Dh * Dv, Dv);               // (r1, r2)
  g.B = P;
  g.bk = imap1(Dn);
  g.bn = imap1(1);
  g.C = Tout + (int64_t)a0 * Dn * Dv * Dv;
  g.cm = imap3(Dv, Dv, (int64_t)Dn * Dv * Dv, Dv, 1);        // (a, u, d)
  g.cn = imap1((int64_t)Dv * Dv);                            // b
  g.alpha = alpha;
  g.beta = beta;
  g.kfast_a = false;
  g.nfast_b = true;
  gemm(g, s);
}

// ---------------------------------------------------------------------------
// one run
// ---------------------------------------------------------------------------

struct Sectors {
  std::vector<int32_t> label, start, n, idx;
};

static Sectors make_sectors(const std::vector<int> &lh, int sym, int q) {
  const int Dh = (int)lh.size();
  std::map<int, std::vector<int32_t>> by;
  for (int a = 0; a < Dh; ++a)
    for (int b = 0; b < Dh; ++b) by[fuse(lh[a], lh[b], sym, q)].push_back(a * Dh + b);
  Sectors s;
  for (auto &kv : by) {
    s.label.push_back(kv.first);
    s.start.push_back((int32_t)s.idx.size());
    s.n.push_back((int32_t)kv.second.size());
    s.idx.insert(s.idx.end(), kv.second.begin(), kv.second.end());
  }
  return s;
}

struct EigMem {
  double *A, *V, *Q, *scale;
  int32_t *flags, *ints;
  int64_t ints_cap, eig_elems, eig_q;
  double *B1, *B2;        // scratch matrices of the refinement stage
  int64_t *gtab;          // offset tables of the batched matrix products
  GGroup *ggrp;
  int64_t gtab_cap, ggrp_cap;
};

// Stage tolerances of the block-Jacobi solver (scale = max |E_ii| of the
// batch). Stage 1 removes couplings above 1e-9 scale. The refinement removes
// couplings above 64 eps scale, and also smaller ones between nearly
// degenerate states whose rotation angle |a_pq / (a_pp - a_qq)| exceeds 1e-6
// (these decide which of two close states is kept at the cut), but never
// couplings below 8 eps sqrt(|a_pp a_qq|), the rounding noise the 32 x 32
// block updates regenerate.
constexpr double kEps = 2.220446049250313e-16;
constexpr double kStage1Abs = 1e-9;
constexpr double kStage2Abs = 64 * kEps;
constexpr double kStage2Rel = 8 * kEps;
constexpr double kStage2Gap = 1e-6;

// Sweeps until no pair has a significant coupling; returns the sweep count.
static int jacobi_sweeps(const EigBatch &eb, double abs_tol, double rel_tol, double gap_tol,
                         hipStream_t s, int32_t *hp) {
  const int nmat = eb.nmat;
  launch_eig_scale(eb, s);
  launch_fill_i32(eb.d_flags + nmat, nmat, 0, s);
  const int max_sweeps = (int)env_size("GXY_JACOBI_MAX_SWEEPS", kMaxSweeps);
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int rr = 0; rr < eb.max_nb - 1; ++rr)
      launch_eig_round(eb, rr, abs_tol, rel_tol, gap_tol, 1, s);
    // flags <- next flags, next <- 0, and read them back
    GXY_HIP(hipMemcpyAsync(eb.d_flags, eb.d_flags + nmat, nmat * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s));
    launch_fill_i32(eb.d_flags + nmat, nmat, 0, s);
    GXY_HIP(hipMemcpyAsync(hp, eb.d_flags, nmat * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GXY_HIP(hipStreamSynchronize(s));
    bool any = false;
    for (int k = 0; k < nmat; ++k) any |= hp[k] != 0;
    if (!any) return sweep + 1;
  }
  fail(GXY_ENUMERIC, "block-Jacobi eigensolver did not converge");
}

struct SectorSolve {
  EigBatch eb;
  const int32_t *d_idx, *d_start, *d_n, *d_lab;
  int sweeps, sweeps2;  // block-Jacobi sweeps of the two stages
  // tridiagonal path: eigenvalues are on diag(eb.A); the vectors are formed by
  // vectors(d_side) once the side is known (d_side null: both sides)
  bool vectors_pending = false;
  int nmat = 0, nsec = 0, kmax = 0, maxn = 0;
  double *Y = nullptr, *work = nullptr;
  void vectors(const double *d_side, hipStream_t s) const {
    if (!vectors_pending) return;
    launch_tri_vectors(nmat, nsec, maxn, d_n, eb.d_npad, eb.d_off, eb.A, eb.V, Y, work, kmax,
                       d_side, s);
  }
};

// Which batched eigensolver: where every sector has at most kTriMaxN rows and
// at most kTriMaxVecs eigenvectors are needed, Householder tridiagonalisation
// + bisection + inverse iteration (O(n^3) once); otherwise block Jacobi
// (O(n^3) per sweep, tens of sweeps). GXY_EIG=jacobi forces block Jacobi.
enum { EIG_AUTO = 0, EIG_JACOBI = 1, EIG_TRI = 2 };
static int eig_method_env() {
  const char *v = getenv("GXY_EIG");
  if (!v) return EIG_AUTO;
  if (!strcmp(v, "jacobi")) return EIG_JACOBI;
  if (!strcmp(v, "tri")) return EIG_TRI;
  return EIG_AUTO;
}

// Eigendecomposition of every label sector of E_L (E) and E_R (E + nf*nf).
// kmax: eigenvectors needed per sector (the leading ones; the tridiagonal
// path forms only those). hp: pinned host scratch (>= 2 * nsec ints).
static SectorSolve solve_sectors(gxy_ctx *ctx, hipStream_t s, const double *E, int nf,
                                 const Sectors &sec, const EigMem &m, int32_t *hp,
                                 int kmax, int method = EIG_AUTO) {
  const int nsec = (int)sec.label.size();
  const int nmat = 2 * nsec;
  std::vector<int32_t> npad(nmat), pairbase(nmat + 1), pair_mat, tiles;
  std::vector<int64_t> off(nmat);
  int64_t tot = 0;
  int max_nb = 2;
  for (int k = 0; k < nmat; ++k) {
    const int nn = sec.n[k % nsec];
    npad[k] = ((nn + 31) / 32) * 32;
    off[k] = tot;
    tot += (int64_t)npad[k] * npad[k];
    const int nb = npad[k] / 16;
    max_nb = std::max(max_nb, nb);
    pairbase[k] = (int32_t)pair_mat.size();
    for (int q = 0; q < nb / 2; ++q) pair_mat.push_back(k);
  }
  pairbase[nmat] = (int32_t)pair_mat.size();
  if (tot > m.eig_elems) fail(GXY_ENOMEM, "eigen workspace bound exceeded");
  if ((int64_t)pair_mat.size() * 1024 > m.eig_q) fail(GXY_ENOMEM, "rotation buffer bound exceeded");
  for (int k = 0; k < nmat; ++k) {
    const int np2 = npad[k] / 32;  // pairs per matrix = row blocks of 32
    for (int x = 0; x < np2; ++x)
      for (int y = x + 1; y < np2; ++y) tiles.insert(tiles.end(), {k, 0, x, y});
    for (int x = 0; x < np2; ++x)
      for (int y = 0; y < np2; ++y) tiles.insert(tiles.end(), {k, 1, x, y});
  }
  // pack: idx | start | n | label | npad | off (2 ints each) | pairbase | pair_mat | tiles
  std::vector<int32_t> pack;
  pack.reserve(sec.idx.size() + 3 * nsec + nmat * 3 + pairbase.size() + pair_mat.size() +
               tiles.size() + 2);
  auto put = [&](const std::vector<int32_t> &v) {
    const size_t at = pack.size();
    pack.insert(pack.end(), v.begin(), v.end());
    return at;
  };
  const size_t o_idx = put(sec.idx), o_start = put(sec.start), o_n = put(sec.n),
               o_lab = put(sec.label), o_npad = put(npad);
  while (pack.size() % 2) pack.push_back(0);
  const size_t o_off = pack.size();
  pack.resize(pack.size() + 2 * nmat);
  memcpy(pack.data() + o_off, off.data(), sizeof(int64_t) * nmat);
  const size_t o_pb = put(pairbase), o_pm = put(pair_mat), o_tl = put(tiles);
  if ((int64_t)pack.size() > m.ints_cap) fail(GXY_ENOMEM, "table workspace bound exceeded");
  GXY_HIP(hipMemcpyAsync(m.ints, pack.data(), pack.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, s));
  SectorSolve r{};
  r.d_idx = m.ints + o_idx;
  r.d_start = m.ints + o_start;
  r.d_n = m.ints + o_n;
  r.d_lab = m.ints + o_lab;
  EigBatch &eb = r.eb;
  eb.nmat = nmat;
  eb.d_npad = m.ints + o_npad;
  eb.d_off = reinterpret_cast<int64_t *>(m.ints + o_off);
  eb.d_pairbase = m.ints + o_pb;
  eb.d_pair_mat = m.ints + o_pm;
  eb.total_pairs = (int32_t)pair_mat.size();
  eb.max_nb = max_nb;
  eb.A = m.A;
  eb.V = m.V;
  eb.Q = m.Q;
  eb.d_flags = m.flags;
  eb.d_scale = m.scale;
  eb.d_rtl = m.ints + o_tl;
  eb.n_update_tiles = (int32_t)(tiles.size() / 4);
  eb.d_pair_rot = m.flags + 2 * nmat;
  int maxn = 0;
  for (int k = 0; k < nsec; ++k) maxn = std::max(maxn, (int)sec.n[k]);
  if (method == EIG_AUTO) method = eig_method_env();
  if (method != EIG_JACOBI && maxn <= kTriMaxN && std::min(kmax, maxn) <= kTriMaxVecs) {
    // Householder tridiagonalisation + bisection now; inverse iteration and
    // back-transformation later, for the chosen side only
    EigBatch eg = eb;
    eg.V = nullptr;
    launch_eig_gather(E, nf, r.d_idx, r.d_start, r.d_n, nsec, eg, s);
    std::vector<int> hn(sec.n.begin(), sec.n.end());
    launch_tri_values(nmat, nsec, hn.data(), r.d_n, eb.d_npad, eb.d_off, m.A, m.B1, m.V, m.B2,
                      !single_stream(ctx), s);
    r.eb.A = m.A;
    r.eb.V = m.V;
    r.sweeps = 0;
    r.sweeps2 = 0;
    r.vectors_pending = true;
    r.nmat = nmat;
    r.nsec = nsec;
    r.maxn = maxn;
    r.kmax = std::max(1, kmax);
    r.Y = m.B1;
    r.work = m.B2;
    return r;
  }
  // batched products over the padded matrices: C = A B and C = A^T B
  TablePlan tp;
  Launch L_nn, L_tn;
  {
    std::vector<GGroup> nn, tn;
    L_nn.first_group = 0;
    for (int k = 0; k < nmat; ++k) {
      const int np = npad[k];
      std::vector<int64_t> R(np), I(np), RT(np), IT(np);
      for (int i = 0; i < np; ++i) {
        R[i] = off[k] + (int64_t)i * np;
        I[i] = i;
        RT[i] = off[k] + i;
        IT[i] = (int64_t)i * np;
      }
      const int64_t oR = (int64_t)tp.tab.size();
      tp.tab.insert(tp.tab.end(), R.begin(), R.end());
      const int64_t oI = (int64_t)tp.tab.size();
      tp.tab.insert(tp.tab.end(), I.begin(), I.end());
      const int64_t oRT = (int64_t)tp.tab.size();
      tp.tab.insert(tp.tab.end(), RT.begin(), RT.end());
      const int64_t oIT = (int64_t)tp.tab.size();
      tp.tab.insert(tp.tab.end(), IT.begin(), IT.end());
      nn.push_back(GGroup{np, np, np, 0, oR, oI, oR, oI, oR, oI});
      tn.push_back(GGroup{np, np, np, 0, oRT, oIT, oR, oI, oR, oI});
    }
    auto finish = [&](std::vector<GGroup> &gs, Launch &L, bool kfa) {
      L.first_group = (int32_t)tp.groups.size();
      L.tile = 64;
      L.kfast_a = kfa;
      L.nfast_b = true;
      for (GGroup g : gs) {
        g.tile_start = L.total_tiles;
        L.total_tiles += ((g.M + 63) / 64) * ((g.N + 63) / 64);
        tp.groups.push_back(g);
        ++L.ngroups;
      }
    };
    finish(nn, L_nn, true);
    finish(tn, L_tn, false);
  }
  upload_plan(ctx, 2, tp, m.gtab, m.gtab_cap, m.ggrp, m.ggrp_cap, s);
  auto mm = [&](const Launch &L, const double *A, const double *B, double *C, double alpha,
                double beta) { run_launch(L, m.ggrp, m.gtab, A, B, C, alpha, beta, s); };

  // stage 1: block Jacobi on the sectors of E to a loose tolerance
  launch_eig_gather(E, nf, r.d_idx, r.d_start, r.d_n, nsec, eb, s);
  r.sweeps = jacobi_sweeps(eb, kStage1Abs, 0.0, 1e300, s, hp);
  // re-orthonormalise the accumulated rotations (one Newton-Schulz step):
  // V2 = V (3 I - V^T V) / 2
  mm(L_tn, m.V, m.V, m.B1, 1.0, 0.0);
  launch_eig_scaled_copy(tot, 1.5, m.V, m.B2, s);
  mm(L_nn, m.V, m.B1, m.B2, -0.5, 1.0);
  // Rayleigh-Ritz with the original sector matrices: R = V2^T E_s V2
  EigBatch e_orig = eb;
  e_orig.A = m.B1;
  e_orig.V = nullptr;
  launch_eig_gather(E, nf, r.d_idx, r.d_start, r.d_n, nsec, e_orig, s);
  mm(L_nn, m.B1, m.B2, m.A, 1.0, 0.0);
  mm(L_tn, m.B2, m.A, m.B1, 1.0, 0.0);
  // stage 2: R is nearly diagonal; Jacobi to rounding level
  EigBatch e2 = eb;
  e2.A = m.B1;
  e2.V = m.A;
  launch_eig_identity(e2, m.A, s);
  r.sweeps2 = jacobi_sweeps(e2, kStage2Abs, kStage2Rel, kStage2Gap, s, hp);
  // eigenvectors V = V2 W, eigenvalues on the diagonal of the final R
  mm(L_nn, m.B2, m.A, m.V, 1.0, 0.0);
  r.eb.A = m.B1;
  r.eb.V = m.V;
  return r;
}

static void run_one(gxy_ctx *ctx, const gxy_point &p, gxy_result &res, RunLog &log) {
  validate(p);
  const hipStream_t s = ctx->stream;
  const size_t chunk_bytes =
      ctx->chunk_bytes ? ctx->chunk_bytes : env_size("GXY_CHUNK_BYTES", kDefaultChunkBytes);
  // batch workers keep to their one stream: many workers already fill the
  // device, and every extra stream shares the few hardware queues
  const Plan pl = make_plan(p, chunk_bytes, !single_stream(ctx));
  const bool gemm_dma = env_flag("GXY_GEMM_DMA");
  Buffers b{};
  {
    Carver c0;
    const size_t need = carve(p, pl, c0, b);
    ensure_workspace(ctx, need);
    Carver c;
    c.base = (char *)ctx->ws;
    carve(p, pl, c, b);
  }
  ensure_pinned(ctx, 1 << 20);
  // impurity stream: the impurity projections of step n run there while the
  // main stream goes on with step n + 1 (its environments and eigensolves
  // leave most compute units idle). Event slots: 0 initial tensors, 1 X of
  // the step ready, 2 norm of the step ready, 3 end of the run, 4 + parity
  // the impurity stream is done with that parity's buffers.
  if (pl.overlap && !ctx->imp_stream)
    GXY_HIP(hipStreamCreateWithFlags(&ctx->imp_stream, hipStreamNonBlocking));
  const hipStream_t si = pl.overlap ? ctx->imp_stream : s;
  struct ImpGuard {
    hipStream_t si, s;
    ~ImpGuard() {
      if (si != s) (void)hipStreamSynchronize(si);
    }
  } impg{si, s};
  auto record_on = [&](hipStream_t st, int slot) {
    if (!ctx->pipe_ev[slot])
      GXY_HIP(hipEventCreateWithFlags(&ctx->pipe_ev[slot], hipEventDisableTiming));
    GXY_HIP(hipEventRecord(ctx->pipe_ev[slot], st));
  };
  Timer tm;
  tm.on = env_flag("GXY_TIMING") && !ctx->noalloc;
  ctx->hot_on = !ctx->noalloc && (tm.on || ctx->hot_force || env_flag("GXY_HOT_EVENTS"));
  ctx->hot_launches.clear();
  tm.s = s;
  tm.acc = ctx->phase_ms;
  for (double &v : ctx->phase_ms) v = 0.0;
  if (tm.on) {
    GXY_HIP(hipEventCreate(&tm.a));
    GXY_HIP(hipEventCreate(&tm.b));
  }
  struct EvGuard {
    Timer &t;
    ~EvGuard() {
      if (t.on) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
      }
    }
  } evg{tm};

  const int sym = sym_of(p);
  const int nmax = p.nmax;
  const int D0 = pl.d0;
  const int qmax = 4 * nmax;
  double *t = b.coef;
  double *F = t + D0;
  double *FM = F + (2 * qmax + 1);
  double *FM1 = FM + (2 * qmax + 1);
  double *FS1 = FM1 + (2 * qmax + 1);   // cos^2 theta
  double *FS2 = FS1 + (2 * qmax + 1);   // cos^2 q theta

  tm.begin();
  const int qh = harmonic(p);
  launch_char_coeffs(p.beta, p.delta, qh, nmax, p.nquad, t, s);
  launch_field_factors(p.beta, p.h, p.h1, qh, qmax, kLmax, sym == SYM_U1, F, FM, FM1, s);
  launch_init_tensor(t, F, nmax, b.T, s);
  const Chains ch = chains_of(p);
  if (p.impurities & (GXY_IMP_COS1_SQ | GXY_IMP_COS2_SQ))
    launch_square_factors(qh, qmax, FS1, FS2, s);
  for (int k = 0; k < ch.n; ++k) {
    const int w = ch.which[k];
    const double *Fk = w == GXY_IMP_COS1 ? FM : w == GXY_IMP_COS2 ? FM1
                       : w == GXY_IMP_COS1_SQ ? FS1 : FS2;
    launch_init_tensor(t, Fk, nmax, b.TX[k], s);
  }
  const int nimp = pl.nimp;
  int Dh = D0, Dv = D0;
  int64_t nT = (int64_t)Dh * Dh * Dv * Dv;
  launch_fro_norm(b.T, nT, b.partial, b.nrm, s);
  launch_scale(b.T, nT, b.nrm + 2, s);
  for (int k = 0; k < nimp; ++k) launch_scale(b.TX[k], nT, b.nrm + 2, s);
  stream_after(ctx, si, s, 0);
  tm.end(0);

  const int mod = (sym == SYM_U1) ? 0 : (sym == SYM_Z2 ? qh : 1);
  // allowed Q = q_l + q_d - q_r - q_u of each impurity tensor (cos theta
  // carries charge +-1, cos q theta +-q; with Z_q labels these are mod q)
  QSet imp_set[4];
  for (int k = 0; k < nimp; ++k) {
    const int w = ch.which[k];
    const bool cos1 = w == GXY_IMP_COS1;
    if (w == GXY_IMP_COS1_SQ)          // zero field only: cos^2 carries 0, +-2
      imp_set[k] = QSet{-2, 0, 2};
    else if (w == GXY_IMP_COS2_SQ)     // cos^2 q: 0, +-2q
      imp_set[k] = QSet{-2 * qh, 0, 2 * qh};
    else if (sym == SYM_U1)
      imp_set[k] = cos1 ? QSet{-1, 1} : QSet{-qh, qh};
    else if (sym == SYM_Z2)
      imp_set[k] = cos1 ? qset_sum(QSet{1, -1}, QSet{0}, qh) : QSet{0};
    else
      imp_set[k] = QSet{0};
  }
  std::vector<int> lh(D0), lv(D0);
  for (int i = 0; i < D0; ++i) {
    const int c = i - nmax;
    lh[i] = lv[i] = (sym == SYM_U1) ? c : (sym == SYM_Z2 ? (((c % qh) + qh) % qh) : 0);
  }
  log.steps.clear();
  res.near_ties = 0;
  res.max_trunc_err = 0.0;
  res.min_cut_gap = INFINITY;

  int32_t *hp = ctx->noalloc ? (int32_t *)ctx->noalloc_host : (int32_t *)ctx->pinned;
  const int inject_nan_step = (int)env_size("GXY_INJECT_NAN_STEP", 0);
  // the next step's environment tables, planned on a host thread as soon as
  // this step's kept labels are known (used only if the legs it was planned
  // for are the next step's)
  struct EnvPlan {
    int Dh = 0, Dv = 0;
    std::vector<int> lh, lv;
    TablePlan tp;
    Launch le[3], re[3];
  };
  std::future<std::shared_ptr<EnvPlan>> env_next;
  for (int n = 1; n <= p.nsteps; ++n) {
    const StepDims &sd = pl.steps[n - 1];
    // buffers of this step's parity; the impurity stream read them last in
    // step n - 2
    const int par = n & 1;
    // host arena of the step's tables: by parity with the impurity stream,
    // else one (single-stream runs drain it before reuse)
    const int aq = pl.overlap ? par : 0;
    b.P = b.Pb[par];
    b.X = b.Xb[par];
    b.T2 = b.T2b[par];
    b.perm = b.permb[par];
    b.proj_tab = b.tabb[par];
    if (si != s && n > 2) GXY_HIP(hipStreamWaitEvent(s, ctx->pipe_ev[4 + par], 0));
    if (sd.xstep) {
      // T[l][r][u][d] -> T[u][d][l][r]
      tm.begin();
      launch_swap_pairs(b.T, b.Tn, Dh, Dh, Dv, Dv, s);
      std::swap(b.T, b.Tn);
      for (int k = 0; k < nimp; ++k) {
        launch_swap_pairs(b.TX[k], b.TXn[k], Dh, Dh, Dv, Dv, si);
        std::swap(b.TX[k], b.TXn[k]);
      }
      std::swap(Dh, Dv);
      std::swap(lh, lv);
      for (int k = 0; k < nimp; ++k) imp_set[k] = qset_negate(imp_set[k], mod);
      tm.end(5);
    }
    const int64_t nf = (int64_t)Dh * Dh;
    const int Dn = sd.dn;
    gxy_step_info info{};
    // precision schedule: the first fp64_steps steps contract in FP64, the
    // rest in the requested form (environments and eigensolves always FP64)
    const int sprec = (n <= p.fp64_steps) ? (int)GXY_PREC_FP64 : (int)p.prec;
    std::vector<int> new_lh;
    if (nf <= p.dcut) {
      launch_identity(b.P, (int)nf, s);
      new_lh.resize(nf);
      for (int a = 0; a < Dh; ++a)
        for (int c = 0; c < Dh; ++c) new_lh[a * Dh + c] = fuse(lh[a], lh[c], sym, qh);
      info.truncated = 0;
    } else {
      // ---- environments ----
      tm.begin();
      if (sym == SYM_NONE) {
        env_gemms(b.T, Dh, Dv, b.envA, b.envB, b.E, false, s);
        env_gemms(b.T, Dh, Dv, b.envA, b.envB, b.E + nf * nf, true, s);
      } else {
        std::shared_ptr<EnvPlan> ep;
        if (env_next.valid()) ep = env_next.get();
        if (!ep || ep->Dh != Dh || ep->Dv != Dv || ep->lh != lh || ep->lv != lv) {
          ep = std::make_shared<EnvPlan>();
          StepLegs SL{Dh, Dv, Dn, mod, lh, lv, {}};
          plan_env(SL, false, ep->tp, ep->le);
          plan_env(SL, true, ep->tp, ep->re);
        }
        const TablePlan &tp = ep->tp;
        const Launch *le = ep->le, *re = ep->re;
        upload_plan(ctx, 0, tp, b.tab_env, pl.tab_env, b.grp_env, pl.grp_env, s);
        run_launch(le[0], b.grp_env, b.tab_env, b.T, b.T, b.envA, 1.0, 0.0, s);
        run_launch(le[1], b.grp_env, b.tab_env, b.T, b.T, b.envB, 1.0, 0.0, s);
        run_launch(le[2], b.grp_env, b.tab_env, b.envA, b.envB, b.E, 1.0, 0.0, s);
        run_launch(re[0], b.grp_env, b.tab_env, b.T, b.T, b.envA, 1.0, 0.0, s);
        run_launch(re[1], b.grp_env, b.tab_env, b.T, b.T, b.envB, 1.0, 0.0, s);
        run_launch(re[2], b.grp_env, b.tab_env, b.envA, b.envB, b.E + nf * nf, 1.0, 0.0, s);
      }
      tm.end(1);
      // ---- sectors and eigensolver tables ----
      tm.begin();
      const Sectors sec = make_sectors(lh, sym, qh);
      const int nsec = (int)sec.label.size();
      EigMem em{b.eigA, b.eigV, b.eigQ, b.eig_scale, b.eig_flags, b.ints, b.ints_cap,
                b.eig_elems, b.eig_q, b.eigB1, b.eigB2, b.gtab, b.ggrp, b.gtab_cap,
                b.ggrp_cap};
      const SectorSolve sv = solve_sectors(ctx, s, b.E, (int)nf, sec, em, hp, Dn);
      const EigBatch &eb = sv.eb;
      info.eig_sweeps = sv.sweeps + 100 * sv.sweeps2;
      const int32_t *d_idx = sv.d_idx, *d_start = sv.d_start, *d_n = sv.d_n,
                    *d_lab = sv.d_lab;
      tm.end(2);
      // ---- truncation ----
      tm.begin();
      SelectArgs sa{};
      sa.nsec = nsec;
      sa.d_sec_label = d_lab;
      sa.d_sec_n = d_n;
      sa.d_mat_off = eb.d_off;
      sa.d_mat_npad = eb.d_npad;
      sa.A = eb.A;
      sa.dcut = Dn;
      sa.ncand = (int32_t)nf;
      sa.tie_rel = kTieRel;
      sa.side_tol = kSideTol;
      sa.d_lam = b.sel_lam;
      sa.d_cand_sec = b.sel_int;
      sa.d_cand_rank = b.sel_int + 2 * nf;
      sa.d_cand_col = b.sel_int + 4 * nf;
      sa.d_taken = b.sel_int + 6 * nf;
      sa.d_pick_sec = b.pick;
      sa.d_pick_col = b.pick + Dn;
      sa.d_pick_label = b.pick + 2 * Dn;
      sa.d_diag = b.diag;
      launch_select(sa, s);
      // the host needs only the kept labels and the summary; it plans the
      // projection while the device forms the kept eigenvectors and P
      GXY_HIP(hipMemcpyAsync(hp, b.pick + 2 * Dn, Dn * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      double *hd = reinterpret_cast<double *>(hp + 512);
      GXY_HIP(hipMemcpyAsync(hd, b.diag, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
      if (!ctx->noalloc) {
        if (!ctx->sel_ev) GXY_HIP(hipEventCreateWithFlags(&ctx->sel_ev, hipEventDisableTiming));
        GXY_HIP(hipEventRecord(ctx->sel_ev, s));
      }
      sv.vectors(b.diag + 2, s);   // diag[2] = chosen side
      launch_build_projector(eb.V, eb.d_off, eb.d_npad, d_idx, d_start, d_n, b.pick,
                             b.pick + Dn, b.diag, nsec, (int)nf, Dn, b.P, s);
      if (ctx->noalloc)
        GXY_HIP(hipStreamSynchronize(s));
      else
        GXY_HIP(hipEventSynchronize(ctx->sel_ev));
      new_lh.assign(hp, hp + Dn);
      info.eps_l = hd[0];
      info.eps_r = hd[1];
      info.side = (int)hd[2];
      info.lam_max = hd[3];
      info.cut_gap = hd[4];
      info.ties = (int)hd[5];
      info.truncated = 1;
      const double trE = hd[6];
      if (!isfinite(info.lam_max) || !isfinite(trE) || !isfinite(info.eps_l) ||
          !isfinite(info.eps_r)) {
        // the environments of this step are not finite: the run stops here
        res.fail_step = n;
        res.nsteps_done = n - 1;
        fail(GXY_ENUMERIC, "non-finite environment spectrum at step " + std::to_string(n));
      }
      const double eps = info.side ? info.eps_r : info.eps_l;
      if (trE > 0) res.max_trunc_err = std::max(res.max_trunc_err, eps / trE);
      res.min_cut_gap = std::min(res.min_cut_gap, info.cut_gap);
      res.near_ties += info.ties;
      tm.end(3);
    }
    if (sym != SYM_NONE && n < p.nsteps) {
      // the legs the next step's environments will see: this step's output
      // (back in y-orientation after an x-step), then the next step's own
      // transposition
      auto ep = std::make_shared<EnvPlan>();
      ep->Dh = Dn;
      ep->Dv = Dv;
      ep->lh = new_lh;
      ep->lv = lv;
      if (sd.xstep) {
        std::swap(ep->Dh, ep->Dv);
        std::swap(ep->lh, ep->lv);
      }
      if (pl.steps[n].xstep) {
        std::swap(ep->Dh, ep->Dv);
        std::swap(ep->lh, ep->lv);
      }
      const int md = mod;
      env_next = std::async(std::launch::async, [ep, md]() {
        StepLegs SL{ep->Dh, ep->Dv, 0, md, ep->lh, ep->lv, {}};
        plan_env(SL, false, ep->tp, ep->le);
        plan_env(SL, true, ep->tp, ep->re);
        return ep;
      });
    }
    // the new pure tensor's norm and scaling, on the main stream: issued as
    // soon as its last product is, so that the main stream goes on while the
    // host issues the impurity stream's launches
    bool normed = false;
    auto normalise = [&]() {
      if (normed) return;
      normed = true;
      const int64_t nTo = (int64_t)Dn * Dn * Dv * Dv;
      launch_fro_norm(b.Tn, nTo, b.partial, b.nrm + 3 * n, s);
      launch_scale(b.Tn, nTo, b.nrm + 3 * n + 2, s);
      // test hook of the failure path: one NaN planted after step n's
      // normalisation (GXY_INJECT_NAN_STEP = n)
      if (inject_nan_step == n) launch_fill(b.Tn, 1, NAN, s);
    };
    // ---- projection T' = P^T M P (and impurities), chunked over a ----
    tm.begin();
    // bottom operands of the D^7 product: dense path [l][u][r][d]; charge
    // blocks: both fused indices in block order (see plan.h)
    StepLegs blk{Dh, Dv, 0, mod, lh, lv, {}};
    if (sym == SYM_NONE) {
      launch_swap_middle(b.T, b.T2, Dh, Dh, Dv, Dv, s);
      for (int k = 0; k < nimp; ++k) launch_swap_middle(b.TX[k], b.TX2[k], Dh, Dh, Dv, Dv, s);
    } else {
      block_positions(blk);
      const int64_t Wn = (int64_t)Dh * Dv;
      if (Wn > pl.maxW) fail(GXY_ENOMEM, "block order table bound");
    }
    const int64_t per_a = (int64_t)Dh * Dv * Dh * Dv;
    const int ac_max = (int)std::max<int64_t>(1, std::min<int64_t>(Dn, pl.chunk_elems / per_a));
    const double W = (double)Dh * Dv;
    auto hot_y = [&](const double *Xp, const double *Bp, int ac) {
      // algorithmic work of the dense product: 2 M N K flops, A + B + C bytes
      const double M = (double)ac * W;
      hot_begin(ctx, s, 2.0 * M * W * W, 8.0 * (M * W + W * W + M * W));
      proj_y(Xp, Bp, Dh, Dv, ac, b.Y, s, sprec);
      hot_end(ctx, s);
    };
    if (sym == SYM_NONE) {
      for (int a0 = 0; a0 < Dn; a0 += ac_max) {
        const int ac = std::min(ac_max, Dn - a0);
        proj_x(b.P, Dh, Dv, Dn, a0, ac, b.T, b.X, s, sprec);
        hot_y(b.X, b.T2, ac);
        proj_t(b.Y, b.P, Dh, Dv, Dn, a0, ac, 1.0, 0.0, b.Tn, s, sprec);
        for (int k = 0; k < nimp; ++k) {
          hot_y(b.X, b.TX2[k], ac);
          proj_t(b.Y, b.P, Dh, Dv, Dn, a0, ac, 0.5, 0.0, b.TXn[k], s, sprec);
          proj_x(b.P, Dh, Dv, Dn, a0, ac, b.TX[k], b.XI, s, sprec);
          hot_y(b.XI, b.T2, ac);
          proj_t(b.Y, b.P, Dh, Dv, Dn, a0, ac, 0.5, 1.0, b.TXn[k], s, sprec);
        }
      }
    } else {
      // charge-block launches. Every launch of the step is planned on a host
      // thread of its own (at most kPlanAhead ahead of the one the stream
      // needs next) and staged in the pinned arena; the stream takes each as
      // soon as it is ready, so the device runs one launch while the host
      // plans the next.
      ProjArena arena;
      proj_stage_begin(ctx, aq, arena, pl.proj_bytes, pl.maxW, s);
      if (!ctx->copy_stream && !single_stream(ctx))
        GXY_HIP(hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking));
      // this step's table copies overwrite slices of the device area that
      // earlier launches of the compute stream read (the same area every
      // step without the impurity stream): the copy stream starts after them
      if (!single_stream(ctx)) stream_after(ctx, ctx->copy_stream, s, 6);
      // (proj_stage_begin has seen the last launches that read this
      // parity's device slices complete, two steps ago, so the side stream
      // may overwrite them)
      int proj_tile = ctx->force_tile;
      if (!proj_tile) {
        const char *ev = getenv("GXY_PROJ_TILE");
        const int t = ev ? atoi(ev) : 0;
        if (t == 64 || t == 128 || t == 256) proj_tile = t;
      }
      if (!proj_tile) {
        const auto it = ctx->tile_for_dcut.find(p.dcut);
        if (it != ctx->tile_for_dcut.end()) proj_tile = it->second;
      }
      StepLegs SL{Dh, Dv, Dn, mod, lh, lv, new_lh, proj_tile};
      SL.pos = blk.pos;
      SL.vrank = blk.vrank;
      const QSet s0{0};
      // launch kinds: pure X, Y, T'; impurity Y = X(T) T_X2, X(T_X),
      // Y += X(T_X) T2, T' of the summed Y (the projection is linear in Y, so
      // the two placements share one T' product)
      // second-moment chains also Y += 2 X(T1) T1 (the pairs split between
      // the halves), with X(T1) formed again: IX3, IY3
      enum { PX, PY, PT, IY, IX2, IY2, IX3, IY3A, IY3B, IT, NKIND };
      struct Part {
        int a0 = 0, ac = 0, k = -1;  // k = -1: pure tensor; else impurity k
        ProjJob job[NKIND];
      };
      std::vector<Part> parts;
      for (int a0 = 0; a0 < Dn; a0 += ac_max)
        for (int k = -1; k < nimp; ++k) {
          Part pt;
          pt.a0 = a0;
          pt.ac = std::min(ac_max, Dn - a0);
          pt.k = k;
          parts.push_back(pt);
        }
      int last_pure = -1;   // the part with the pure tensor's last products
      for (int i = 0; i < (int)parts.size(); ++i)
        if (parts[i].k < 0) last_pure = i;
      // jobs in the order the stream consumes them
      std::vector<std::pair<int, int>> order;
      for (int i = 0; i < (int)parts.size(); ++i) {
        if (parts[i].k < 0)
          for (int kd : {PX, PY, PT}) order.push_back({i, kd});
        else if (ch.first[parts[i].k] < 0)
          for (int kd : {IY, IX2, IY2, IT}) order.push_back({i, kd});
        else
          for (int kd : {IY, IX2, IY2, IX3, IY3A, IY3B, IT}) order.push_back({i, kd});
      }
      auto plan_job = [&SL, &s0, &imp_set, &parts, &arena, &ch](int i, int kd) {
        Part &pt = parts[i];
        const int a0 = pt.a0, a1 = pt.a0 + pt.ac;
        const QSet &sk = pt.k < 0 ? s0 : imp_set[pt.k];
        const QSet &s1 = (pt.k < 0 || ch.first[pt.k] < 0) ? s0 : imp_set[ch.first[pt.k]];
        TablePlan tp;
        Launch L;
        switch (kd) {
          case PX: L = plan_proj_x(SL, a0, a1, s0, tp); break;
          case PY: L = plan_proj_y(SL, a0, a1, s0, s0, tp); break;
          case PT: L = plan_proj_t(SL, a0, a1, s0, tp); break;
          case IY: L = plan_proj_y(SL, a0, a1, s0, sk, tp); break;
          case IT: L = plan_proj_t(SL, a0, a1, sk, tp); break;
          case IX2: L = plan_proj_x(SL, a0, a1, sk, tp); break;
          case IX3: L = plan_proj_x(SL, a0, a1, s1, tp); break;
          // X(T1) T1 by the charge of the upper factor (U(1): {-c, +c})
          case IY3A: L = plan_proj_y(SL, a0, a1, QSet{s1.front()}, s1, tp); break;
          case IY3B: L = plan_proj_y(SL, a0, a1, QSet{s1.back()}, s1, tp); break;
          default: L = plan_proj_y(SL, a0, a1, sk, s0, tp); break;
        }
        stage_plan(arena, tp, L, pt.job[kd]);
      };
      // declared after everything the threads use, so that unwinding joins
      // them first
      std::vector<std::future<void>> planned(order.size());
      size_t spawned = 0;
      auto spawn_upto = [&](size_t n) {
        for (; spawned < std::min(n, order.size()); ++spawned) {
          const auto o = order[spawned];
          planned[spawned] = std::async(std::launch::async, plan_job, o.first, o.second);
        }
      };
      spawn_upto(kPlanAhead);
      {
        // block-order bottom operands; the permutation is staged in the
        // arena, whose previous copies have completed
        const int64_t Wn = (int64_t)Dh * Dv;
        for (int64_t f = 0; f < Wn; ++f) arena.perm[blk.pos[f]] = (int32_t)f;
        GXY_HIP(hipMemcpyAsync(b.perm, arena.perm, Wn * sizeof(int32_t), hipMemcpyHostToDevice,
                               s));
        if (ctx->noalloc) GXY_HIP(hipStreamSynchronize(s));
        launch_block_gather(b.T, b.T2, b.perm, Dh, Dv, s);
      }
      const int64_t nTn = (int64_t)Dn * Dn * Dv * Dv;
      launch_fill(b.Tn, nTn, 0.0, s);
      // the impurity stream's share (once it has the step's X, T2, P, perm)
      bool imp_started = false;
      auto imp_start = [&]() {
        if (imp_started) return;
        imp_started = true;
        stream_after(ctx, si, s, 1);
        for (int k = 0; k < nimp; ++k) launch_block_gather(b.TX[k], b.TX2[k], b.perm, Dh, Dv, si);
        for (int k = 0; k < nimp; ++k) launch_fill(b.TXn[k], nTn, 0.0, si);
      };
      size_t next = 0;
      auto take = [&](int i, int kd) -> ProjJob & {
        // jobs are consumed in spawn order
        while (next < order.size() && (order[next].first < i ||
                                       (order[next].first == i && order[next].second <= kd))) {
          spawn_upto(next + 1 + kPlanAhead);
          planned[next].get();
          ++next;
        }
        return parts[i].job[kd];
      };
      auto go = [&](ProjJob &j, const double *A, const double *B, double *C, double alpha,
                    double beta, bool hot, hipStream_t st, size_t slot) {
        send_plan(ctx, arena, j, b.proj_tab, st, slot);
        const GGroup *dg = reinterpret_cast<const GGroup *>(b.proj_tab + j.off);
        const int64_t *dt = reinterpret_cast<const int64_t *>(b.proj_tab + j.off +
                                                              j.ngrp * (int64_t)sizeof(GGroup));
        if (hot) hot_begin(ctx, st, j.L.flops, j.L.bytes + (beta != 0.0 ? j.L.c_bytes : 0.0));
        run_launch(j.L, dg, dt, A, B, C, alpha, beta, st, sprec, gemm_dma);
        if (hot) hot_end(ctx, st);
      };
      // (with chunks, both streams are the main one: the next chunk's X
      // overwrites the X the impurity launches read)
      for (int i = 0; i < (int)parts.size(); ++i) {
        const int k = parts[i].k;
        const size_t sl = (size_t)i * NKIND;
        if (k < 0) {
          go(take(i, PX), b.P, b.T, b.X, 1.0, 0.0, false, s, sl + PX);
          go(take(i, PY), b.X, b.T2, b.Y, 1.0, 0.0, true, s, sl + PY);
          go(take(i, PT), b.Y, b.P, b.Tn, 1.0, 0.0, false, s, sl + PT);
          // the impurity launches start once the pure tensor's are issued:
          // the pure products then run without them (Dcut = 64 with both
          // chains: the same steps/s either way, and the D^7 launches
          // average 3.3 ms instead of 4.0)
          if (nimp > 0) imp_start();
          if (i == last_pure) normalise();
        } else {
          // (both Y products write the same blocks: those whose row and
          // column charges differ by a charge of the impurity)
          go(take(i, IY), b.X, b.TX2[k], b.YI, 1.0, 0.0, true, si, sl + IY);
          go(take(i, IX2), b.P, b.TX[k], b.XI, 1.0, 0.0, false, si, sl + IX2);
          go(take(i, IY2), b.XI, b.T2, b.YI, 1.0, 1.0, true, si, sl + IY2);
          const int k1 = ch.first[k];
          if (k1 >= 0) {
            // second moment: (T2 (x) T + T (x) T2 + 2 T1 (x) T1) / 4 with the
            // step's input T1 (its chain wrote only TXn[k1] so far)
            go(take(i, IX3), b.P, b.TX[k1], b.XI, 1.0, 0.0, false, si, sl + IX3);
            go(take(i, IY3A), b.XI, b.TX2[k1], b.YI, 2.0, 1.0, true, si, sl + IY3A);
            go(take(i, IY3B), b.XI, b.TX2[k1], b.YI, 2.0, 1.0, true, si, sl + IY3B);
          }
          go(take(i, IT), b.YI, b.P, b.TXn[k], k1 >= 0 ? 0.25 : 0.5, 0.0, false, si, sl + IT);
        }
      }
      if (si != s) record_on(si, 4 + par);
    }
    tm.end(4);
    tm.begin();
    Dh = Dn;
    nT = (int64_t)Dh * Dh * Dv * Dv;
    normalise();
    std::swap(b.T, b.Tn);
    stream_after(ctx, si, s, 2);
    for (int k = 0; k < nimp; ++k) {
      launch_scale(b.TXn[k], nT, b.nrm + 3 * n + 2, si);
      std::swap(b.TX[k], b.TXn[k]);
    }
    // the step's tables have been read by both streams' launches once the
    // impurity stream gets here
    if (sym != SYM_NONE) proj_stage_done(ctx, aq, si);
    lh = new_lh;
    if (sd.xstep) {
      launch_swap_pairs(b.T, b.Tn, Dh, Dh, Dv, Dv, s);
      std::swap(b.T, b.Tn);
      for (int k = 0; k < nimp; ++k) {
        launch_swap_pairs(b.TX[k], b.TXn[k], Dh, Dh, Dv, Dv, si);
        std::swap(b.TX[k], b.TXn[k]);
      }
      std::swap(Dh, Dv);
      std::swap(lh, lv);
      for (int k = 0; k < nimp; ++k) imp_set[k] = qset_negate(imp_set[k], mod);
    }
    tm.end(5);
    info.dh = Dh;
    info.dv = Dv;
    log.steps.push_back(info);
  }
  // ---- trace and result ----
  stream_after(ctx, s, si, 3);
  // traces at scal[0] (pure) and scal[1 + k] (chain k); results at scal[8..15]
  double *tr = b.scal, *tr1 = b.scal + 1, *rr = b.scal + 8;
  launch_trace(b.T, Dh, Dv, tr, s);
  const double *trk[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int k = 0; k < nimp; ++k) {
    launch_trace(b.TX[k], Dh, Dv, tr1 + k, s);
    const int w = ch.which[k];
    trk[w == GXY_IMP_COS1 ? 0 : w == GXY_IMP_COS2 ? 1 : w == GXY_IMP_COS1_SQ ? 2 : 3] = tr1 + k;
  }
  // lnc[n] lives at nrm[3n + 1]; gather them contiguously into the partial buffer
  GXY_HIP(hipMemcpy2DAsync(b.partial, sizeof(double), b.nrm + 1, 3 * sizeof(double),
                           sizeof(double), p.nsteps + 1, hipMemcpyDeviceToDevice, s));
  launch_finish(b.partial, p.nsteps, p.beta, tr, trk, rr, s);
  double *hd = reinterpret_cast<double *>(hp);
  GXY_HIP(hipMemcpyAsync(hd, rr, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
  GXY_HIP(hipMemcpyAsync(hd + 8, b.partial, (p.nsteps + 1) * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  hot_collect(ctx);
  res.lnz_per_site = hd[0];
  res.m_cos1 = hd[1];
  res.m_cos2 = hd[2];
  res.status = (int32_t)hd[3];
  if (res.status) {
    // the first step whose norm is not finite, else the final trace
    res.fail_step = p.nsteps;
    for (int n = 1; n <= p.nsteps; ++n)
      if (!isfinite(hd[8 + n])) {
        res.fail_step = n;
        break;
      }
  } else {
    res.fail_step = -1;
  }
  res.msq_cos1 = hd[4];
  res.msq_cos2 = hd[5];
  res.chi0 = hd[6];
  res.chi0_n = hd[7];
  res.nsteps_done = p.nsteps;
  if (!isfinite(res.min_cut_gap)) res.min_cut_gap = 0.0;
  for (int n = 1; n <= p.nsteps; ++n) log.steps[n - 1].lnc = hd[8 + n];
}

static void initial_tensor_only(gxy_ctx *ctx, const gxy_point &p, int which, double *out) {
  validate(p);
  const hipStream_t s = ctx->stream;
  const int D0 = 2 * p.nmax + 1, qmax = 4 * p.nmax;
  const int64_t n4 = (int64_t)D0 * D0 * D0 * D0;
  const size_t need = sizeof(double) * (n4 + D0 + 3 * (2 * qmax + 1)) + 4096;
  ensure_workspace(ctx, need);
  double *T = (double *)ctx->ws;
  double *t = T + n4;
  double *F = t + D0, *FM = F + (2 * qmax + 1), *FM1 = FM + (2 * qmax + 1);
  launch_char_coeffs(p.beta, p.delta, harmonic(p), p.nmax, p.nquad, t, s);
  launch_field_factors(p.beta, p.h, p.h1, harmonic(p), qmax, kLmax, sym_of(p) == SYM_U1, F, FM,
                       FM1, s);
  launch_init_tensor(t, which == 0 ? F : (which == 1 ? FM : FM1), p.nmax, T, s);
  GXY_HIP(hipMemcpyAsync(out, T, n4 * sizeof(double), hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
}

static size_t workspace_for(const gxy_point &p) {
  validate(p);
  const Plan pl = make_plan(p, env_size("GXY_CHUNK_BYTES", kDefaultChunkBytes));
  Buffers b{};
  Carver c;
  return carve(p, pl, c, b);
}

// ---------------------------------------------------------------------------
// no-allocation runs: a fixed device scratch array
// ---------------------------------------------------------------------------

// Device memory of gxy_run_noalloc. Host code never uses this name as an
// address (on the host it is only a stand-in): each device's copy is found
// with hipGetSymbolAddress at gxy_create and kept in the context.
constexpr size_t kScratchBytes = GXY_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// The scratch address on `device`, which must be current; looked up once
// per device.
static void *scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) fail(GXY_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    GXY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(GXY_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

// Largest projection chunk bound whose workspace fits the scratch array
// (0 if none does).
static size_t noalloc_chunk(const gxy_point &p, size_t *need_out) {
  size_t need = 0;
  for (size_t chunk = kDefaultChunkBytes; chunk >= ((size_t)1 << 16); chunk /= 2) {
    const Plan pl = make_plan(p, chunk, false);
    Buffers b{};
    Carver c;
    need = carve(p, pl, c, b);
    if (need <= kScratchBytes) {
      *need_out = need;
      return chunk;
    }
  }
  *need_out = need;
  return 0;
}

// Routes the context's runs through the scratch array for one call and
// restores its own workspace afterwards.
struct NoallocScope {
  gxy_ctx *ctx;
  void *ws;
  size_t ws_bytes, chunk;
  bool owned;
  NoallocScope(gxy_ctx *c, size_t chunk_bytes)
      : ctx(c), ws(c->ws), ws_bytes(c->ws_bytes), chunk(c->chunk_bytes), owned(c->ws_owned) {
    c->ws = c->scratch;
    c->ws_bytes = kScratchBytes;
    c->ws_owned = false;
    c->chunk_bytes = chunk_bytes;
    c->noalloc = true;
  }
  ~NoallocScope() {
    ctx->ws = ws;
    ctx->ws_bytes = ws_bytes;
    ctx->ws_owned = owned;
    ctx->chunk_bytes = chunk;
    ctx->noalloc = false;
  }
};

}  // namespace gxy

// ===========================================================================
// C ABI
// ===========================================================================

using gxy::Error;


extern "C" {

gxy_status gxy_create(gxy_ctx **out, int device, void *hip_stream) {
  if (!out) return GXY_EINVAL;
  *out = nullptr;
  gxy_ctx *ctx = nullptr;
  GXY_API_BEGIN
  int n = 0;
  GXY_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return GXY_EINVAL;
  GXY_HIP(hipSetDevice(device));
  ctx = new gxy_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  try {
    ctx->scratch = gxy::scratch_address(device);
  } catch (...) {
    delete ctx;
    ctx = nullptr;
    throw;
  }
  *out = ctx;
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_destroy(gxy_ctx *ctx) {
  if (!ctx) return GXY_EINVAL;
  (void)hipSetDevice(ctx->device);
  for (gxy_ctx *c : ctx->children) {
    hipStream_t cs = c->stream;
    gxy_destroy(c);
    if (cs) (void)hipStreamDestroy(cs);
  }
  ctx->children.clear();
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->imp_stream) (void)hipStreamSynchronize(ctx->imp_stream);
  if (ctx->copy_stream) (void)hipStreamSynchronize(ctx->copy_stream);
  if (ctx->ws && ctx->ws_owned) (void)hipFree(ctx->ws);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (int q = 0; q < 2; ++q) {
    if (ctx->arena_ev[q]) (void)hipEventDestroy(ctx->arena_ev[q]);
    if (ctx->arena[q] && !ctx->arena_pageable[q]) (void)hipHostFree(ctx->arena[q]);
  }
  for (hipEvent_t e : ctx->pipe_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->imp_stream) (void)hipStreamDestroy(ctx->imp_stream);
  if (ctx->sel_ev) (void)hipEventDestroy(ctx->sel_ev);
  for (hipEvent_t e : ctx->copy_ev) (void)hipEventDestroy(e);
  if (ctx->copy_stream) (void)hipStreamDestroy(ctx->copy_stream);
  for (int j = 0; j < 3; ++j) {
    if (ctx->stage_ev[j]) (void)hipEventDestroy(ctx->stage_ev[j]);
    if (ctx->stage[j]) (void)hipHostFree(ctx->stage[j]);
  }
  delete ctx;
  return GXY_OK;
}

gxy_status gxy_workspace_bytes(gxy_ctx *ctx, const gxy_point *pts, int32_t n, size_t *bytes) {
  if (!ctx || !pts || n <= 0 || !bytes) return GXY_EINVAL;
  GXY_API_BEGIN
  size_t m = 0;
  for (int i = 0; i < n; ++i) m = std::max(m, gxy::workspace_for(pts[i]));
  *bytes = m;
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_set_workspace(gxy_ctx *ctx, void *dev_ptr, size_t bytes) {
  if (!ctx) return GXY_EINVAL;
  if (dev_ptr && bytes == 0) return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  if (ctx->ws && ctx->ws_owned) GXY_HIP(hipFree(ctx->ws));
  ctx->ws = dev_ptr;
  ctx->ws_bytes = dev_ptr ? bytes : 0;
  ctx->ws_owned = false;
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_char_coeffs(gxy_ctx *ctx, double beta, double delta, int32_t nmax,
                           int32_t nquad, double *t) {
  if (!ctx || !t || nmax < 0 || nmax > 64 || nquad <= 2 * nmax || !(beta >= 0.0) ||
      !(delta >= 0.0 && delta <= 1.0))
    return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  gxy::ensure_workspace(ctx, sizeof(double) * (2 * nmax + 1) + 256);
  double *d = (double *)ctx->ws;
  gxy::launch_char_coeffs(beta, delta, 2, nmax, nquad, d, ctx->stream);
  GXY_HIP(hipMemcpyAsync(t, d, sizeof(double) * (2 * nmax + 1), hipMemcpyDeviceToHost,
                         ctx->stream));
  GXY_HIP(hipStreamSynchronize(ctx->stream));
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_initial_tensor(gxy_ctx *ctx, const gxy_point *pt, int32_t which, double *out) {
  if (!ctx || !pt || !out || which < 0 || which > 2) return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  gxy::initial_tensor_only(ctx, *pt, which, out);
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_run(gxy_ctx *ctx, const gxy_point *pt, gxy_result *out) {
  if (!ctx || !pt || !out) return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  ctx->logs.assign(1, gxy::RunLog{});
  gxy_result r{};
  r.status = GXY_OK;
  r.fail_step = -1;
  try {
    gxy::run_one(ctx, *pt, r, ctx->logs[0]);
  } catch (const Error &e) {
    if (e.status != GXY_ENUMERIC) throw;
    // a numerical failure during the run: the result names the step
    r.status = e.status;
    r.lnz_per_site = r.m_cos1 = r.m_cos2 = NAN;
    r.msq_cos1 = r.msq_cos2 = r.chi0 = r.chi0_n = NAN;
    *out = r;
    throw;
  }
  *out = r;
  if (r.status) ctx->last_error = "non-finite result (first failing step " +
                                  std::to_string(r.fail_step) + ")";
  return (gxy_status)r.status;
  GXY_API_END(ctx)
}

gxy_status gxy_run_noalloc(gxy_ctx *ctx, const gxy_point *pt, gxy_result *out) {
  if (!ctx || !pt || !out) return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  gxy::validate(*pt);
  if (!ctx->scratch) gxy::fail(GXY_EDEVICE, "no scratch address on this device");
  size_t need = 0;
  const size_t chunk = gxy::noalloc_chunk(*pt, &need);
  if (!chunk)
    gxy::fail(GXY_EINVAL, "the run needs " + std::to_string(need) +
                              " bytes of device workspace; gxy_run_noalloc holds at most " +
                              std::to_string(gxy::kScratchBytes));
  gxy::NoallocScope scope(ctx, chunk);
  ctx->logs.assign(1, gxy::RunLog{});
  gxy_result r{};
  r.status = GXY_OK;
  r.fail_step = -1;
  gxy::run_one(ctx, *pt, r, ctx->logs[0]);
  *out = r;
  return (gxy_status)r.status;
  GXY_API_END(ctx)
}

gxy_status gxy_run_batch(gxy_ctx *ctx, const gxy_point *pts, int32_t n, gxy_result *out) {
  if (!ctx || !pts || !out || n <= 0) return GXY_EINVAL;
  try {
    GXY_HIP(hipSetDevice(ctx->device));
  } catch (const Error &e) {
    ctx->last_error = e.msg;
    return e.status;
  }
  int W = ctx->batch_workers;
  if (W <= 0) W = (int)gxy::env_size("GXY_BATCH_WORKERS", 4);
  W = std::max(1, std::min(W, n));
  std::vector<gxy::RunLog> logs(n);
  for (int i = 0; i < n; ++i) {
    out[i] = gxy_result{};
    out[i].fail_step = -1;
  }
  std::atomic<bool> dead{false};
  std::mutex err_mu;
  std::string last;
  // one run on context c; a device error stops the whole batch
  auto one = [&](gxy_ctx *c, int i) {
    gxy_result r{};
    r.fail_step = -1;
    try {
      GXY_HIP(hipSetDevice(c->device));
      gxy::run_one(c, pts[i], r, logs[i]);
    } catch (const Error &e) {
      r.status = e.status;
      r.lnz_per_site = r.m_cos1 = r.m_cos2 = NAN;
      r.msq_cos1 = r.msq_cos2 = r.chi0 = r.chi0_n = NAN;
      std::lock_guard<std::mutex> g(err_mu);
      last = e.msg;
      if (e.status == GXY_EDEVICE) dead = true;
    } catch (...) {
      r.status = GXY_EDEVICE;
      r.lnz_per_site = r.m_cos1 = r.m_cos2 = NAN;
      r.msq_cos1 = r.msq_cos2 = r.chi0 = r.chi0_n = NAN;
      std::lock_guard<std::mutex> g(err_mu);
      last = "unexpected host exception";
      dead = true;
    }
    out[i] = r;
  };
  if (W == 1) {
    for (int i = 0; i < n && !dead; ++i) one(ctx, i);
  } else {
    try {
      // worker contexts: own non-blocking stream (default priority), the
      // parent's tile table, ordered after the work already on its stream
      while ((int)ctx->children.size() < W) {
        hipStream_t cs = nullptr;
        GXY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        gxy_ctx *c = new gxy_ctx();
        c->device = ctx->device;
        c->stream = cs;
        c->chunk_bytes = (size_t)4 << 30;   // smaller projection chunks per worker
        c->worker = true;
        ctx->children.push_back(c);
      }
      hipEvent_t ev = nullptr;
      GXY_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      GXY_HIP(hipEventRecord(ev, ctx->stream));
      for (int w = 0; w < W; ++w) {
        ctx->children[w]->tile_for_dcut = ctx->tile_for_dcut;
        ctx->children[w]->force_tile = ctx->force_tile;
        GXY_HIP(hipStreamWaitEvent(ctx->children[w]->stream, ev, 0));
      }
      GXY_HIP(hipEventDestroy(ev));
    } catch (const Error &e) {
      ctx->last_error = e.msg;
      return e.status;
    }
    // longest runs first (cost ~ Dcut^7 per placement, dense steps dearer)
    std::vector<int> order(n);
    std::vector<double> cost(n);
    for (int i = 0; i < n; ++i) {
      const gxy_point &p = pts[i];
      const int nimp = gxy::chains_of(p).n;
      const double D = std::max(1, std::min(p.dcut, 128));
      cost[i] = std::pow(D, 7.0) * std::max(p.nsteps, 1) * (1 + 2 * nimp) *
                ((p.h != 0.0) ? 16.0 : (p.h1 != 0.0 ? 2.0 : 1.0));
      order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return cost[a] > cost[b]; });
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    for (int w = 0; w < W; ++w)
      th.emplace_back([&, w]() {
        gxy_ctx *c = ctx->children[w];
        for (;;) {
          if (dead) return;
          const int k = next++;
          if (k >= n) return;
          one(c, order[k]);
        }
      });
    for (auto &t : th) t.join();
    for (int w = 0; w < W; ++w) (void)hipStreamSynchronize(ctx->children[w]->stream);
  }
  ctx->logs = std::move(logs);
  bool any_fail = false;
  for (int i = 0; i < n; ++i) {
    if (dead && out[i].status == GXY_OK && out[i].nsteps_done == 0 && pts[i].nsteps > 0) {
      out[i].status = GXY_EDEVICE;
      out[i].lnz_per_site = out[i].m_cos1 = out[i].m_cos2 = NAN;
      out[i].msq_cos1 = out[i].msq_cos2 = out[i].chi0 = out[i].chi0_n = NAN;
    }
    any_fail |= out[i].status != GXY_OK;
  }
  if (!last.empty()) ctx->last_error = last;
  if (dead) return GXY_EDEVICE;
  return any_fail ? GXY_EPARTIAL : GXY_OK;
}

gxy_status gxy_set_batch_workers(gxy_ctx *ctx, int32_t workers) {
  if (!ctx || workers < 0 || workers > 64) return GXY_EINVAL;
  ctx->batch_workers = workers;
  return GXY_OK;
}

gxy_status gxy_autotune(gxy_ctx *ctx, const gxy_point *templ, const int32_t *dcuts, int32_t n,
                        int32_t *tiles, double *ms) {
  if (!ctx || !templ || !dcuts || n <= 0) return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  for (int i = 0; i < n; ++i) {
    gxy_point p = *templ;
    p.dcut = dcuts[i];
    gxy::validate(p);
    double best_ms = 0.0;
    int best = 0;
    const int cand[3] = {64, 128, 256};
    for (int ti = 0; ti < 3; ++ti) {
      const int tile = cand[ti];
      ctx->force_tile = tile;
      ctx->hot_force = true;
      double st[4] = {0, 0, 0, 0};
      ctx->logs.assign(1, gxy::RunLog{});
      gxy_result r{};
      r.fail_step = -1;
      try {
        // first run warms the code objects and the workspace, second is timed
        gxy::run_one(ctx, p, r, ctx->logs[0]);
        for (int j = 0; j < 4; ++j) ctx->hot_stats[j] = 0.0;
        gxy::run_one(ctx, p, r, ctx->logs[0]);
      } catch (...) {
        ctx->force_tile = 0;
        ctx->hot_force = false;
        throw;
      }
      for (int j = 0; j < 4; ++j) st[j] = ctx->hot_stats[j];
      if (ms) ms[3 * i + ti] = st[1];
      if (best == 0 || st[1] < best_ms) {
        best = tile;
        best_ms = st[1];
      }
    }
    ctx->force_tile = 0;
    ctx->hot_force = false;
    for (int j = 0; j < 4; ++j) ctx->hot_stats[j] = 0.0;
    ctx->tile_for_dcut[p.dcut] = best;
    if (tiles) tiles[i] = best;
  }
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_step_log(gxy_ctx *ctx, int32_t run, gxy_step_info *out, int32_t cap,
                        int32_t *count) {
  if (!ctx || !count || run < 0 || run >= (int32_t)ctx->logs.size() || cap < 0 ||
      (cap > 0 && !out))
    return GXY_EINVAL;
  const auto &st = ctx->logs[run].steps;
  const int32_t m = std::min<int32_t>(cap, (int32_t)st.size());
  for (int i = 0; i < m; ++i) out[i] = st[i];
  *count = (int32_t)st.size();
  return GXY_OK;
}

gxy_status gxy_observables(gxy_ctx *ctx, int32_t npts, const double *beta, const double *lnz,
                           const double *m_h, const double *m_h1, double dbeta, double dh,
                           double dh1, double *out) {
  if (!ctx || npts <= 0 || !beta || !lnz || !m_h || !m_h1 || !out || !(dbeta > 0) ||
      !(dh > 0) || !(dh1 > 0))
    return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  const size_t n = (size_t)npts;
  const size_t need = sizeof(double) * (n + 3 * n + 2 * n + 2 * n + 4 * n) + 1024;
  gxy::ensure_workspace(ctx, need);
  double *d = (double *)ctx->ws;
  double *db = d, *dl = db + n, *dm = dl + 3 * n, *dm1 = dm + 2 * n, *dout = dm1 + 2 * n;
  hipStream_t s = ctx->stream;
  GXY_HIP(hipMemcpyAsync(db, beta, n * sizeof(double), hipMemcpyHostToDevice, s));
  GXY_HIP(hipMemcpyAsync(dl, lnz, 3 * n * sizeof(double), hipMemcpyHostToDevice, s));
  GXY_HIP(hipMemcpyAsync(dm, m_h, 2 * n * sizeof(double), hipMemcpyHostToDevice, s));
  GXY_HIP(hipMemcpyAsync(dm1, m_h1, 2 * n * sizeof(double), hipMemcpyHostToDevice, s));
  gxy::launch_observables(npts, db, dl, dm, dm1, dbeta, dh, dh1, dout, s);
  GXY_HIP(hipMemcpyAsync(out, dout, 4 * n * sizeof(double), hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  return GXY_OK;
  GXY_API_END(ctx)
}

static int64_t lgt_links_of(int32_t ndim, const int32_t *dims, int64_t nconf) {
  int64_t V = 1;
  for (int mu = 0; mu < ndim; ++mu) V *= dims[mu];
  return nconf * ndim * V;
}

static bool lgt_args_ok(int32_t ndim, const int32_t *dims, int64_t nconf, uint32_t flags) {
  if (!dims || ndim < 2 || ndim > 4 || nconf < 0 || nconf > GXY_LGT_MAX_CONF ||
      (flags & ~(uint32_t)GXY_LGT_FULL) != 0)
    return false;
  int64_t V = 1;
  for (int mu = 0; mu < ndim; ++mu) {
    if (dims[mu] < 2) return false;   // a plaquette needs four distinct links
    V *= dims[mu];
    if (V > INT32_MAX) return false;
  }
  return true;
}

gxy_status gxy_lgt_workspace_bytes(int32_t ndim, const int32_t *dims, int64_t nconf,
                                   uint32_t flags, size_t *out) {
  if (!out || !lgt_args_ok(ndim, dims, nconf, flags)) return GXY_EINVAL;
  *out = gxy::lgt_workspace_doubles(ndim, dims, nconf, (flags & GXY_LGT_FULL) != 0) *
             sizeof(double) + 1024;
  return GXY_OK;
}

gxy_status gxy_lgt_estimator(gxy_ctx *ctx, const double *theta, int32_t ndim,
                             const int32_t *dims, int64_t nconf, uint32_t flags,
                             gxy_lgt_result *out) {
  if (!ctx || !lgt_args_ok(ndim, dims, nconf, flags) || (nconf > 0 && (!theta || !out)))
    return GXY_EINVAL;
  if (nconf == 0) return GXY_OK;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  const bool full = (flags & GXY_LGT_FULL) != 0;
  const size_t nd = gxy::lgt_workspace_doubles(ndim, dims, nconf, full);
  gxy::ensure_workspace(ctx, nd * sizeof(double) + 1024);
  double *ws = (double *)ctx->ws;
  double *dres = ws + nd - (size_t)nconf * 14;
  hipStream_t s = ctx->stream;
  // GXY_HOT_EVENTS: events around the gradient kernel, with its algorithmic
  // bytes (every link's U read once, g written once with GXY_LGT_FULL)
  ctx->hot_on = !ctx->noalloc && gxy::env_flag("GXY_HOT_EVENTS");
  struct HotArg {
    gxy_ctx *ctx;
    double bytes;
  } ha{ctx, (double)lgt_links_of(ndim, dims, nconf) * (full ? 24.0 : 16.0)};
  gxy::LgtHooks hooks{[](void *a, hipStream_t st) {
                        auto *h = static_cast<HotArg *>(a);
                        gxy::hot_begin(h->ctx, st, 0.0, h->bytes);
                      },
                      [](void *a, hipStream_t st) {
                        gxy::hot_end(static_cast<HotArg *>(a)->ctx, st);
                      },
                      &ha};
  gxy::lgt_estimate(theta, ndim, dims, nconf, full, ws, dres, s, ctx->hot_on ? &hooks : nullptr);
  static_assert(sizeof(gxy_lgt_result) == 14 * sizeof(double), "result layout");
  GXY_HIP(hipMemcpyAsync(out, dres, (size_t)nconf * sizeof(gxy_lgt_result),
                         hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  gxy::hot_collect(ctx);
  ctx->hot_on = false;
  return GXY_OK;
  GXY_API_END(ctx)
}

const char *gxy_status_string(gxy_status s) {
  switch (s) {
    case GXY_OK: return "ok";
    case GXY_EINVAL: return "invalid argument";
    case GXY_ENOMEM: return "out of device memory";
    case GXY_EDEVICE: return "HIP runtime error";
    case GXY_ENUMERIC: return "numerical failure";
    case GXY_EUNSUPPORTED: return "unsupported request";
    case GXY_EPARTIAL: return "some runs of the batch failed";
  }
  return "unknown status";
}

const char *gxy_last_error(gxy_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

gxy_status gxy_hot_kernel_stats(gxy_ctx *ctx, double *out4, int32_t reset) {
  if (!ctx || !out4) return GXY_EINVAL;
  for (int i = 0; i < 4; ++i) out4[i] = ctx->hot_stats[i];
  if (reset)
    for (double &v : ctx->hot_stats) v = 0.0;
  return GXY_OK;
}

gxy_status gxy_phase_times(gxy_ctx *ctx, double *ms6) {
  if (!ctx || !ms6) return GXY_EINVAL;
  for (int i = 0; i < 6; ++i) ms6[i] = ctx->phase_ms[i];
  return GXY_OK;
}

}  // extern "C"

// ===========================================================================
// unit-test entry points (include/gxy_hotrg_testing.h)
// ===========================================================================

extern "C" {

gxy_status gxy_test_gemm(gxy_ctx *ctx, int32_t prec, int32_t M, int32_t N, int32_t K,
                         const double *A, int32_t a_trans, const double *B, int32_t b_trans,
                         double *Cout) {
  if (!ctx || M <= 0 || N <= 0 || K < 0 || !A || !B || !Cout) return GXY_EINVAL;
  if (prec < GXY_PREC_FP64 || prec > GXY_PREC_BF16X3) return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  const size_t na = (size_t)M * K, nb = (size_t)K * N, nc = (size_t)M * N;
  gxy::ensure_workspace(ctx, sizeof(double) * (na + nb + nc) + 1024);
  double *dA = (double *)ctx->ws, *dB = dA + na, *dC = dB + nb;
  hipStream_t s = ctx->stream;
  GXY_HIP(hipMemcpyAsync(dA, A, na * sizeof(double), hipMemcpyHostToDevice, s));
  GXY_HIP(hipMemcpyAsync(dB, B, nb * sizeof(double), hipMemcpyHostToDevice, s));
  gxy::GemmDesc g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = dA;
  g.B = dB;
  g.C = dC;
  g.alpha = 1.0;
  g.beta = 0.0;
  g.am = a_trans ? gxy::imap1(1) : gxy::imap1(K);
  g.ak = a_trans ? gxy::imap1(M) : gxy::imap1(1);
  g.kfast_a = !a_trans;
  g.bk = b_trans ? gxy::imap1(1) : gxy::imap1(N);
  g.bn = b_trans ? gxy::imap1(K) : gxy::imap1(1);
  g.nfast_b = !b_trans;
  g.cm = gxy::imap1(N);
  g.cn = gxy::imap1(1);
  g.prec = prec;
  gxy::gemm(g, s);
  GXY_HIP(hipMemcpyAsync(Cout, dC, nc * sizeof(double), hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_test_gemm_f64(gxy_ctx *ctx, int32_t M, int32_t N, int32_t K, const double *A,
                             int32_t a_trans, const double *B, int32_t b_trans, double *Cout) {
  return gxy_test_gemm(ctx, GXY_PREC_FP64, M, N, K, A, a_trans, B, b_trans, Cout);
}

gxy_status gxy_test_eigh(gxy_ctx *ctx, int32_t n, const double *A, double *w, double *V,
                         int32_t *sweeps) {
  return gxy_test_eigh_method(ctx, 0, n, A, w, V, sweeps);
}

gxy_status gxy_test_eigh_method(gxy_ctx *ctx, int32_t method, int32_t n, const double *A,
                                double *w, double *V, int32_t *sweeps) {
  return gxy_test_eigh_top(ctx, method, n, n, A, w, V, sweeps);
}

gxy_status gxy_test_eigh_top(gxy_ctx *ctx, int32_t method, int32_t n, int32_t kmax,
                             const double *A, double *w, double *V, int32_t *sweeps) {
  if (!ctx || n <= 0 || n > 8192 || !A || !w || !V || method < 0 || method > 2 || kmax < 1 ||
      kmax > n)
    return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  using namespace gxy;
  // one sector holding every index, on both "sides" (the second copy is unused)
  Sectors sec;
  sec.label = {0};
  sec.start = {0};
  sec.n = {n};
  sec.idx.resize(n);
  for (int i = 0; i < n; ++i) sec.idx[i] = i;
  const int64_t np = ((n + 31) / 32) * 32;
  const int64_t nn = (int64_t)n * n;
  EigMem m{};
  m.eig_elems = 2 * np * np;
  m.eig_q = 2 * (np / 32) * 1024 + 1024;
  const int64_t tiles = 2 * (3 * (np / 32) * (np / 32) / 2 + 4);
  m.ints_cap = n + 8 + 12 + 4 + 2 * (np / 32) + 4 * tiles + 64;
  m.gtab_cap = 8 * np + 64;
  m.ggrp_cap = 8;
  Carver c;
  for (int pass = 0; pass < 2; ++pass) {
    double *E = c.take<double>(2 * nn);
    m.A = c.take<double>(m.eig_elems);
    m.V = c.take<double>(m.eig_elems);
    m.B1 = c.take<double>(m.eig_elems);
    m.B2 = c.take<double>(m.eig_elems);
    m.gtab = c.take<int64_t>(m.gtab_cap);
    m.ggrp = c.take<GGroup>(m.ggrp_cap);
    m.Q = c.take<double>(m.eig_q);
    m.scale = c.take<double>(8);
    m.flags = c.take<int32_t>(16 + 2 * (np / 32) + 16);
    m.ints = c.take<int32_t>(m.ints_cap);
    if (pass == 0) {
      ensure_workspace(ctx, c.off + 256);
      c = Carver{};
      c.base = (char *)ctx->ws;
      continue;
    }
    ensure_pinned(ctx, 1 << 20);
    hipStream_t s = ctx->stream;
    GXY_HIP(hipMemcpyAsync(E, A, nn * sizeof(double), hipMemcpyHostToDevice, s));
    GXY_HIP(hipMemcpyAsync(E + nn, A, nn * sizeof(double), hipMemcpyHostToDevice, s));
    const SectorSolve sv =
        solve_sectors(ctx, s, E, n, sec, m, (int32_t *)ctx->pinned, kmax, method);
    sv.vectors(nullptr, s);
    if (sweeps) *sweeps = sv.sweeps + sv.sweeps2;
    // eigenvalues: diagonal of the converged matrix; vectors: first n rows/cols
    GXY_HIP(hipMemcpy2DAsync(V, n * sizeof(double), sv.eb.V, np * sizeof(double),
                             n * sizeof(double), n, hipMemcpyDeviceToHost, s));
    GXY_HIP(hipMemcpy2DAsync(w, sizeof(double), sv.eb.A, (np + 1) * sizeof(double),
                             sizeof(double), n, hipMemcpyDeviceToHost, s));
    GXY_HIP(hipStreamSynchronize(s));
  }
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_test_mfma_layout(gxy_ctx *ctx, const double *a, const double *b, double *out) {
  if (!ctx || !a || !b || !out) return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  gxy::ensure_workspace(ctx, sizeof(double) * 384 + 256);
  double *da = (double *)ctx->ws, *db = da + 64, *dout = db + 64;
  hipStream_t s = ctx->stream;
  GXY_HIP(hipMemcpyAsync(da, a, 64 * sizeof(double), hipMemcpyHostToDevice, s));
  GXY_HIP(hipMemcpyAsync(db, b, 64 * sizeof(double), hipMemcpyHostToDevice, s));
  gxy::launch_mfma_probe(da, db, dout, s);
  GXY_HIP(hipMemcpyAsync(out, dout, 256 * sizeof(double), hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_test_mfma_layout32(gxy_ctx *ctx, int32_t kind, const float *a, const float *b,
                                  float *out) {
  if (!ctx || !a || !b || !out || kind < 0 || kind > 1) return GXY_EINVAL;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  const int n = kind == 0 ? 64 : 512;
  gxy::ensure_workspace(ctx, sizeof(float) * (2 * n + 256) + 256);
  float *da = (float *)ctx->ws, *db = da + n, *dout = db + n;
  hipStream_t s = ctx->stream;
  GXY_HIP(hipMemcpyAsync(da, a, n * sizeof(float), hipMemcpyHostToDevice, s));
  GXY_HIP(hipMemcpyAsync(db, b, n * sizeof(float), hipMemcpyHostToDevice, s));
  gxy::launch_mfma_probe32(kind, da, db, dout, s);
  GXY_HIP(hipMemcpyAsync(out, dout, 256 * sizeof(float), hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  return GXY_OK;
  GXY_API_END(ctx)
}

}  // extern "C"
