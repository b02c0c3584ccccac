// Matrix-core GEMMs with index-fused operands for the HOTRG contractions.
//
// Every contraction of a HOTRG step (the environment Gram matrices of the
// mode unfoldings of M, eq. hosvd, and the three factors of the projection
// P^T M P, eqs. Mtensor and renormalizedT) is a matrix product whose row,
// column and reduction indices are fusions of tensor legs. Operands are read
// in place: element (m, k) of A lives at A[row_off(m) + col_off(k)].
//
// Two addressings share one tile body:
//  * affine: mixed-radix index maps (dense contractions);
//  * grouped tables: a launch holds many independent dense sub-products
//    (the charge blocks left by the U(1) or Z2 symmetry of the site tensor),
//    each with its own row / reduction / column offset tables.
//
// Three arithmetic forms share the tile body. Operands and results are FP64
// in memory in every form; the form decides what the matrix cores see:
//  * F64:    v_mfma_f64_16x16x4_f64, FP64 accumulation;
//  * F32:    operands rounded to FP32, v_mfma_f32_16x16x4_f32, FP32
//            accumulation;
//  * BF16X3: operands rounded to FP32 and split x = hi + lo into two bfloat16
//            terms; hi*hi + hi*lo + lo*hi by v_mfma_f32_16x16x32_bf16, FP32
//            accumulation (the lo*lo term is dropped).
//
// Tiling for CDNA4: a workgroup owns a BM x BN output tile; its waves (wave64)
// form a WGM x WGN grid, each wave owning (BM/WGM) x (BN/WGN) built from 16x16
// matrix-core blocks. A and B k-slices are staged through double-buffered LDS
// (one barrier per k-slice). The index tables of the operands are gathered
// one k-slice ahead of the data, so a data load never waits for its own
// address. Workgroups are renumbered so that each XCD (own L2) works on a
// contiguous band of output tiles.
#include <type_traits>

#include "internal.h"

namespace gxy {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

enum { kF64 = GXY_PREC_FP64, kF32 = GXY_PREC_FP32, kB3 = GXY_PREC_BF16X3 };

struct AffineAddr {
  static constexpr bool kContig = false;
  const IdxMap *am, *ak, *bk, *bn, *cm, *cn;
  __device__ int64_t a_m(int m) const { return imap_off(*am, m); }
  __device__ int64_t a_k(int k) const { return imap_off(*ak, k); }
  __device__ int64_t b_k(int k) const { return imap_off(*bk, k); }
  __device__ int64_t b_n(int n) const { return imap_off(*bn, n); }
  __device__ int64_t c_m(int m) const { return imap_off(*cm, m); }
  __device__ int64_t c_n(int n) const { return imap_off(*cn, n); }
};

struct TableAddr {
  static constexpr bool kContig = false;
  const int64_t *ar, *ac, *br, *bc, *cr, *cc;
  __device__ int64_t a_m(int m) const { return ar[m]; }
  __device__ int64_t a_k(int k) const { return ac[k]; }
  __device__ int64_t b_k(int k) const { return br[k]; }
  __device__ int64_t b_n(int n) const { return bc[n]; }
  __device__ int64_t c_m(int m) const { return cr[m]; }
  __device__ int64_t c_n(int n) const { return cc[n]; }
};

// A charge block whose reduction and column indices are contiguous ranges
// (block order): A(m, k) = A[rows[m] + a0 + k], B(k, n) = B[b0 + k ldb + n],
// C(m, n) = C[rows[m] + c0 + n]. Only the rows go through a table.
struct ContigAddr {
  static constexpr bool kContig = true;
  const int64_t *rows;
  int64_t a0, b0, ldb, c0;
  __device__ int64_t a_m(int m) const { return rows[m] + a0; }
  __device__ int64_t a_k(int k) const { return k; }
  __device__ int64_t b_k(int k) const { return b0 + (int64_t)k * ldb; }
  __device__ int64_t b_n(int n) const { return n; }
  __device__ int64_t c_m(int m) const { return rows[m] + c0; }
  __device__ int64_t c_n(int n) const { return n; }
};

// two consecutive doubles, 8-byte aligned (one 16-byte load)
typedef double double2_u __attribute__((ext_vector_type(2), aligned(8)));

// LDS staging of one operand slice (two stages). F64/F32: [k][m] rows with a
// small pad. BF16X3: [k/8][m] cells of 8 consecutive k (one 16-byte read per
// lane feeds a 16x16x32 instruction), hi and lo terms in separate arrays.
template <int BK, int BX, int PREC>
struct Stage {
  double v[2][BK][BX + 2];
  __device__ void put(int st, int k, int x, double a) { v[st][k][x] = a; }
};
template <int BK, int BX>
struct Stage<BK, BX, kF32> {
  float v[2][BK][BX + 4];
  __device__ void put(int st, int k, int x, double a) { v[st][k][x] = (float)a; }
};
template <int BK, int BX>
struct Stage<BK, BX, kB3> {
  bf16x8_t hi[2][BK / 8][BX + 1];
  bf16x8_t lo[2][BK / 8][BX + 1];
  __device__ void put(int st, int k, int x, double a) {
    const float f = (float)a;
    const __bf16 h = (__bf16)f;
    const __bf16 l = (__bf16)(f - (float)h);
    ((__bf16 *)&hi[st][k >> 3][x])[k & 7] = h;
    ((__bf16 *)&lo[st][k >> 3][x])[k & 7] = l;
  }
};

template <int PREC> struct Acc { typedef float4_t type; };
template <> struct Acc<kF64> { typedef double4_t type; };

// The k loop and epilogue shared by every addressing: load(k0) fetches the
// operand slice starting at k0 into registers, store(st) writes it to LDS
// stage st; slices are double-buffered with one barrier per slice.
template <int BM, int BN, int BK, int WGM, int WGN, int PREC, class Addr, class LoadF,
          class StoreF>
__device__ __forceinline__ void gemm_mainloop(const Addr &ad, int M, int N, int K, int m0,
                                              int n0, double *C, double alpha, double beta,
                                              Stage<BK, BM, PREC> &sa, Stage<BK, BN, PREC> &sb,
                                              LoadF &load, StoreF &store, bool mirror = false) {
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm0 = (wave / WGN) * WM;
  const int wn0 = (wave % WGN) * WN;
  typedef typename Acc<PREC>::type acc_t;
  acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  const int ktiles = (K + BK - 1) / BK;
  const int li = lane & 15;
  const int lk = lane >> 4;
  if (ktiles > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int kt = 0; kt < ktiles; ++kt) {
    const int st = kt & 1;
    if (kt + 1 < ktiles) load((kt + 1) * BK);
    if constexpr (PREC == kB3) {
#pragma unroll
      for (int kk = 0; kk < BK / 8; kk += 4) {
        bf16x8_t ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          ah[i] = sa.hi[st][kk + lk][wm0 + 16 * i + li];
          al[i] = sa.lo[st][kk + lk][wm0 + 16 * i + li];
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          bh[j] = sb.hi[st][kk + lk][wn0 + 16 * j + li];
          bl[j] = sb.lo[st][kk + lk][wn0 + 16 * j + li];
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        typedef typename std::remove_reference<decltype(sa.v[0][0][0])>::type op_t;
        op_t fa[FM], fb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) fa[i] = sa.v[st][kk + lk][wm0 + 16 * i + li];
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[j] = sb.v[st][kk + lk][wn0 + 16 * j + li];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if constexpr (PREC == kF64)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
          }
      }
    }
    if (kt + 1 < ktiles) store(st ^ 1);
    __syncthreads();
  }

  // Accumulator register r of lane l holds column l%16 and row l/16 + 4r
  // (FP64 instruction) or 4(l/16) + r (FP32-accumulating instructions).
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int n = n0 + wn0 + 16 * j + li;
    if (n >= N) continue;
    const int64_t noff = ad.c_n(n);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm0 + 16 * i + (PREC == kF64 ? lk + 4 * r : 4 * lk + r);
        if (m >= M) continue;
        double *dst = C + ad.c_m(m) + noff;
        const double v = alpha * (double)acc[i][j][r];
        *dst = (beta == 0.0) ? v : v + beta * (*dst);
        // symmetric launches (beta = 0, M = N): the transposed element, which
        // the tile across the diagonal would compute from the same products
        // in the same order
        if (mirror) C[ad.c_m(n) + ad.c_n(m)] = v;
      }
    }
  }
}

// One BM x BN output tile of C(m, n) = alpha sum_k A(m, k) B(k, n) + beta C.
template <int BM, int BN, int BK, int WGM, int WGN, bool KFA, bool NFB, int PREC, class Addr>
__device__ __forceinline__ void gemm_tile(const Addr &ad, int M, int N, int K, int m0, int n0,
                                          const double *__restrict__ A,
                                          const double *__restrict__ B, double *C,
                                          double alpha, double beta, Stage<BK, BM, PREC> &sa,
                                          Stage<BK, BN, PREC> &sb, bool mirror = false) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_PER = BM * BK / NT, B_PER = BN * BK / NT;
  static_assert(NT % BK == 0 && NT % BM == 0 && NT % BN == 0, "thread mapping");
  static_assert(BM % (NT / BK) == 0 && BN % (NT / BK) == 0, "thread mapping");
  static_assert(BK % (NT / BM) == 0 && BK % (NT / BN) == 0, "thread mapping");
  static_assert(FM >= 1 && FN >= 1 && WM % 16 == 0 && WN % 16 == 0, "wave tile");
  static_assert(PREC != kB3 || BK % 32 == 0, "bf16 k-step");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WGN) * WM;
  const int wn0 = (wave % WGN) * WN;

  // Contiguous reduction and column ranges: each thread moves pairs of
  // consecutive doubles (16-byte loads), A along k and B along n, and no
  // offset table is read inside the k loop.
  constexpr bool CONTIG = Addr::kContig && KFA && NFB;
  constexpr int VA = BK / 2, VB = BN / 2;           // pairs per A row / B row
  constexpr int A_VEC = CONTIG ? BM * VA / NT : 1, B_VEC = CONTIG ? BK * VB / NT : 1;
  static_assert(!CONTIG || (NT % VA == 0 && NT % VB == 0 && BM * VA % NT == 0 &&
                            BK * VB % NT == 0), "pair mapping");
  if constexpr (CONTIG) {
    int64_t arow[A_VEC];
    bool aok[A_VEC];
#pragma unroll
    for (int p = 0; p < A_VEC; ++p) {
      const int m = m0 + tid / VA + (NT / VA) * p;
      aok[p] = m < M;
      arow[p] = aok[p] ? ad.a_m(m) : 0;
    }
    const int ka = 2 * (tid % VA);                  // k of this thread's A pairs
    const int nb = 2 * (tid % VB);                  // n of this thread's B pairs
    const bool nb0 = n0 + nb < N, nb1 = n0 + nb + 1 < N;
    const double *Bc = B + n0 + nb;
    double2_u va[A_VEC], vb[B_VEC];
    auto load_pairs = [&](int k0) {
      const int k = k0 + ka;
#pragma unroll
      for (int p = 0; p < A_VEC; ++p) {
        const double *src = A + arow[p] + k;
        if (aok[p] && k + 1 < K)
          va[p] = *reinterpret_cast<const double2_u *>(src);
        else
          va[p] = double2_u{(aok[p] && k < K) ? src[0] : 0.0, 0.0};
      }
#pragma unroll
      for (int p = 0; p < B_VEC; ++p) {
        const int kb = k0 + tid / VB + (NT / VB) * p;
        const double *src = Bc + ad.b_k(kb);
        if (kb < K && nb1)
          vb[p] = *reinterpret_cast<const double2_u *>(src);
        else
          vb[p] = double2_u{(kb < K && nb0) ? src[0] : 0.0, 0.0};
      }
    };
    auto store_pairs = [&](int st) {
#pragma unroll
      for (int p = 0; p < A_VEC; ++p) {
        const int m = tid / VA + (NT / VA) * p;
        sa.put(st, ka, m, va[p].x);
        sa.put(st, ka + 1, m, va[p].y);
      }
#pragma unroll
      for (int p = 0; p < B_VEC; ++p) {
        const int kb = tid / VB + (NT / VB) * p;
        sb.put(st, kb, nb, vb[p].x);
        sb.put(st, kb, nb + 1, vb[p].y);
      }
    };
    gemm_mainloop<BM, BN, BK, WGM, WGN, PREC>(ad, M, N, K, m0, n0, C, alpha, beta, sa, sb,
                                              load_pairs, store_pairs);
  } else {
  // fixed (row / column) parts of the operand offsets of this thread
  int64_t a_fixed[KFA ? A_PER : 1];
  bool a_ok[KFA ? A_PER : 1];
  if (KFA) {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      const int m = m0 + tid / BK + (NT / BK) * p;
      a_ok[p] = m < M;
      a_fixed[p] = a_ok[p] ? ad.a_m(m) : 0;
    }
  } else {
    const int m = m0 + tid % BM;
    a_ok[0] = m < M;
    a_fixed[0] = a_ok[0] ? ad.a_m(m) : 0;
  }
  int64_t b_fixed[NFB ? 1 : B_PER];
  bool b_ok[NFB ? 1 : B_PER];
  if (NFB) {
    const int n = n0 + tid % BN;
    b_ok[0] = n < N;
    b_fixed[0] = b_ok[0] ? ad.b_n(n) : 0;
  } else {
#pragma unroll
    for (int p = 0; p < B_PER; ++p) {
      const int n = n0 + tid / BK + (NT / BK) * p;
      b_ok[p] = n < N;
      b_fixed[p] = b_ok[p] ? ad.b_n(n) : 0;
    }
  }

  // reduction-index parts, gathered one slice ahead (-1 = beyond K)
  constexpr int TA = KFA ? 1 : A_PER, TB = NFB ? B_PER : 1;
  int64_t ta[TA], tb[TB];
  auto load_offsets = [&](int k0) {
    if (KFA) {
      const int k = k0 + tid % BK;
      ta[0] = k < K ? ad.a_k(k) : -1;
    } else {
#pragma unroll
      for (int p = 0; p < A_PER; ++p) {
        const int k = k0 + tid / BM + (NT / BM) * p;
        ta[p] = k < K ? ad.a_k(k) : -1;
      }
    }
    if (NFB) {
#pragma unroll
      for (int p = 0; p < B_PER; ++p) {
        const int k = k0 + tid / BN + (NT / BN) * p;
        tb[p] = k < K ? ad.b_k(k) : -1;
      }
    } else {
      const int k = k0 + tid % BK;
      tb[0] = k < K ? ad.b_k(k) : -1;
    }
  };
  double ra[A_PER], rb[B_PER];
  auto load_data = [&]() {
    if (KFA) {
#pragma unroll
      for (int p = 0; p < A_PER; ++p)
        ra[p] = (ta[0] >= 0 && a_ok[p]) ? A[a_fixed[p] + ta[0]] : 0.0;
    } else {
#pragma unroll
      for (int p = 0; p < A_PER; ++p)
        ra[p] = (ta[p] >= 0 && a_ok[0]) ? A[a_fixed[0] + ta[p]] : 0.0;
    }
    if (NFB) {
#pragma unroll
      for (int p = 0; p < B_PER; ++p)
        rb[p] = (tb[p] >= 0 && b_ok[0]) ? B[tb[p] + b_fixed[0]] : 0.0;
    } else {
#pragma unroll
      for (int p = 0; p < B_PER; ++p)
        rb[p] = (tb[0] >= 0 && b_ok[p]) ? B[tb[0] + b_fixed[p]] : 0.0;
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      if (KFA)
        sa.put(st, tid % BK, tid / BK + (NT / BK) * p, ra[p]);
      else
        sa.put(st, tid / BM + (NT / BM) * p, tid % BM, ra[p]);
    }
#pragma unroll
    for (int p = 0; p < B_PER; ++p) {
      if (NFB)
        sb.put(st, tid / BN + (NT / BN) * p, tid % BN, rb[p]);
      else
        sb.put(st, tid % BK, tid / BK + (NT / BK) * p, rb[p]);
    }
  };

  auto load_slice = [&](int k0) {
    load_data();
    load_offsets(k0 + BK);
  };
  if (K > 0) load_offsets(0);
  gemm_mainloop<BM, BN, BK, WGM, WGN, PREC>(ad, M, N, K, m0, n0, C, alpha, beta, sa, sb,
                                            load_slice, store, mirror);
  }
}

__device__ __forceinline__ int xcd_remap(int pid, int total) {
  return ((total & 7) == 0) ? (pid & 7) * (total >> 3) + (pid >> 3) : pid;
}

template <int BM, int BN, int BK, int WGM, int WGN, bool KFA, bool NFB, int PREC>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_kernel(GemmDesc g) {
  __shared__ Stage<BK, BM, PREC> sa;
  __shared__ Stage<BK, BN, PREC> sb;
  const int tiles_m = (g.M + BM - 1) / BM;
  const int tiles_n = (g.N + BN - 1) / BN;
  const int total = tiles_m * tiles_n;
  const int pid = xcd_remap(blockIdx.x, total);
  constexpr int GROUP = 8;
  const int in_group = GROUP * tiles_n;
  const int gid = pid / in_group;
  const int first_m = gid * GROUP;
  const int gsize = min(tiles_m - first_m, GROUP);
  const int tm = first_m + (pid % in_group) % gsize;
  const int tn = (pid % in_group) / gsize;
  AffineAddr ad{&g.am, &g.ak, &g.bk, &g.bn, &g.cm, &g.cn};
  gemm_tile<BM, BN, BK, WGM, WGN, KFA, NFB, PREC>(ad, g.M, g.N, g.K, tm * BM, tn * BN, g.A, g.B,
                                                  g.C, g.alpha, g.beta, sa, sb);
}

template <int BM, int BN, int BK, int WGM, int WGN, bool KFA, bool NFB, int PREC>
__global__ __launch_bounds__(64 * WGM * WGN) void ggemm_kernel(GroupedGemm g) {
  __shared__ Stage<BK, BM, PREC> sa;
  __shared__ Stage<BK, BN, PREC> sb;
  const int t = xcd_remap(blockIdx.x, g.total_tiles);
  // group of tile t: last group whose tile_start <= t
  int lo = 0, hi = g.ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.groups[mid].tile_start <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GGroup G = g.groups[lo];
  const int local = t - G.tile_start;
  const int tiles_n = (G.N + BN - 1) / BN;
  int tm = local / tiles_n, tn = local % tiles_n;
  if (g.sym) {
    // row-major lower triangle: tile (tm, tn), tn <= tm, is number
    // tm (tm + 1) / 2 + tn
    tm = (int)((sqrt(8.0 * local + 1.0) - 1.0) * 0.5);
    while (tm * (tm + 1) / 2 > local) --tm;
    while ((tm + 1) * (tm + 2) / 2 <= local) ++tm;
    tn = local - tm * (tm + 1) / 2;
  }
  TableAddr ad{g.tab + G.ar, g.tab + G.ac, g.tab + G.br, g.tab + G.bc, g.tab + G.cr,
               g.tab + G.cc};
  gemm_tile<BM, BN, BK, WGM, WGN, KFA, NFB, PREC>(ad, G.M, G.N, G.K, tm * BM, tn * BN, g.A, g.B,
                                                  g.C, g.alpha, g.beta, sa, sb,
                                                  g.sym && tm != tn);
}

// Grouped launch of contiguous charge blocks (GroupedGemm::contig): group
// fields ar = row table, ac = A column base, br = B base, bc = B row stride,
// cc = C column base.
template <int BM, int BN, int BK, int WGM, int WGN, int PREC>
__global__ __launch_bounds__(64 * WGM * WGN) void ggemm_contig_kernel(GroupedGemm g) {
  __shared__ Stage<BK, BM, PREC> sa;
  __shared__ Stage<BK, BN, PREC> sb;
  const int t = xcd_remap(blockIdx.x, g.total_tiles);
  int lo = 0, hi = g.ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.groups[mid].tile_start <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GGroup G = g.groups[lo];
  const int local = t - G.tile_start;
  const int tiles_n = (G.N + BN - 1) / BN;
  const int tm = local / tiles_n, tn = local % tiles_n;
  ContigAddr ad{g.tab + G.ar, G.ac, G.br, G.bc, G.cc};
  gemm_tile<BM, BN, BK, WGM, WGN, true, true, PREC>(ad, G.M, G.N, G.K, tm * BM, tn * BN, g.A, g.B,
                                                    g.C, g.alpha, g.beta, sa, sb);
}

// FP64 contiguous groups with direct global -> LDS loads (global_load_lds).
//
// A k-slice of 8 is staged as 1 KiB chunks, one per 16 rows of A or 16
// columns of B. Byte 16 l of a chunk holds the two values lane l feeds to
// two consecutive matrix-core steps: A(m, k0 + 2g) and A(m, k0 + 2g + 1) for
// row m = l % 16 of the chunk and lane group g = l / 16, likewise
// B(k0 + 2g, n) and B(k0 + 2g + 1, n). The first step of a slice thus sums
// the even k of the slice and the second the odd ones, and one 16-byte LDS
// read per lane feeds both. The values never pass through registers on the
// way in: an A pair is contiguous in its row and arrives by one 16-byte
// load per lane; a B pair spans two rows, so a B chunk is four 4-byte loads
// per lane (lane i of load j fetches half i % 2 of B(k0 + 2j + (i % 4) / 2,
// n0 + i / 4)). Two stages: the loads of slice t + 1 fly while slice t is
// multiplied. When K is not a multiple of 8 the last slice goes through
// registers, with zeros past K; rows past M and columns past N load the
// last valid row or column (their results are never stored), so every load
// stays inside the group's operands. Every tile shape uses the same slices
// and step order, so the tile does not change the bits.
typedef double double2_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) void lds_void_t;

template <int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void ggemm_dma_kernel(GroupedGemm g) {
  constexpr int NW = WGM * WGN, WM = BM / WGM, WN = BN / WGN, FM = WM / 16, FN = WN / 16;
  constexpr int BK = 8, CA = BM / 16, CB = BN / 16;   // chunks of A and of B per slice
  constexpr int PA = CA / NW, PB = CB / NW;           // chunks each wave fills
  static_assert(CA % NW == 0 && CB % NW == 0 && PA >= 1 && PB >= 1, "chunks per wave");
  static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile");
  __shared__ __attribute__((aligned(1024))) double lds[2][CA + CB][128];
  const int t = xcd_remap(blockIdx.x, g.total_tiles);
  int lo = 0, hi = g.ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.groups[mid].tile_start <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GGroup G = g.groups[lo];
  const int local = t - G.tile_start;
  const int tiles_n = (G.N + BN - 1) / BN;
  const int m0 = (local / tiles_n) * BM, n0 = (local % tiles_n) * BN;
  const int M = G.M, N = G.N, K = G.K;
  const int64_t *rows = g.tab + G.ar;
  const int64_t ldb = G.bc;
  const double *B = g.B + G.br;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;
  const int li = lane & 15, lg = lane >> 4;

  const double *arow[PA];
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    const int m = min(m0 + 16 * (wave + NW * p) + li, M - 1);
    arow[p] = g.A + rows[m] + G.ac + 2 * lg;
  }
  const char *bsrc[PB];
  int bcol[PB];
#pragma unroll
  for (int p = 0; p < PB; ++p) {
    const int c = wave + NW * p;
    bsrc[p] = reinterpret_cast<const char *>(B + ((lane & 3) >> 1) * ldb +
                                             min(n0 + 16 * c + (lane >> 2), N - 1)) +
              4 * (lane & 1);
    bcol[p] = min(n0 + 16 * c + li, N - 1);
  }
  const int ktiles = (K + BK - 1) / BK, kfull = K / BK;
  auto issue = [&](int kt, int st) {
    const int k0 = kt * BK;
    if (kt < kfull) {
#pragma unroll
      for (int p = 0; p < PA; ++p)
        __builtin_amdgcn_global_load_lds((const void *)(arow[p] + k0),
                                         (lds_void_t *)&lds[st][wave + NW * p][0],
                                         16, 0, 0);
#pragma unroll
      for (int p = 0; p < PB; ++p) {
        const char *b = bsrc[p] + (int64_t)k0 * ldb * 8;
        char *dst = reinterpret_cast<char *>(&lds[st][CA + wave + NW * p][0]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          __builtin_amdgcn_global_load_lds((const void *)(b + j * 16 * ldb),
                                           (lds_void_t *)(dst + 256 * j), 4, 0, 0);
      }
    } else {
      const int k = k0 + 2 * lg;
#pragma unroll
      for (int p = 0; p < PA; ++p) {
        const double *a = arow[p] + k0;
        *reinterpret_cast<double2_t *>(&lds[st][wave + NW * p][2 * lane]) =
            double2_t{k < K ? a[0] : 0.0, k + 1 < K ? a[1] : 0.0};
      }
#pragma unroll
      for (int p = 0; p < PB; ++p) {
        const double *b = B + (int64_t)k * ldb + bcol[p];
        *reinterpret_cast<double2_t *>(&lds[st][CA + wave + NW * p][2 * lane]) =
            double2_t{k < K ? b[0] : 0.0, k + 1 < K ? b[ldb] : 0.0};
      }
    }
  };

  double4_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = double4_t{0, 0, 0, 0};
  if (ktiles > 0) issue(0, 0);
  for (int kt = 0; kt < ktiles; ++kt) {
    // every load of slice kt (own and register-path LDS writes) has landed,
    // and every wave is done reading the stage the next loads overwrite
    __builtin_amdgcn_s_waitcnt(0x70);   // vmcnt(0) lgkmcnt(0)
    asm volatile("s_barrier" ::: "memory");
    if (kt + 1 < ktiles) issue(kt + 1, (kt + 1) & 1);
    const int st = kt & 1;
    double2_t fa[FM], fb[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
      fa[i] = *reinterpret_cast<const double2_t *>(&lds[st][wm0 / 16 + i][2 * lane]);
#pragma unroll
    for (int j = 0; j < FN; ++j)
      fb[j] = *reinterpret_cast<const double2_t *>(&lds[st][CA + wn0 / 16 + j][2 * lane]);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].x, fb[j].x, acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].y, fb[j].y, acc[i][j], 0, 0, 0);
  }

  // register r of lane l: row l / 16 + 4 r, column l % 16 of the 16 x 16 block
  const double alpha = g.alpha, beta = g.beta;
  double *C = g.C + G.cc;
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int n = n0 + wn0 + 16 * j + li;
    if (n >= N) continue;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm0 + 16 * i + lg + 4 * r;
        if (m >= M) continue;
        double *dst = C + rows[m] + n;
        const double v = alpha * acc[i][j][r];
        *dst = (beta == 0.0) ? v : v + beta * (*dst);
      }
    }
  }
}

template <int BM, int BN, int WGM, int WGN>
void launch_dma(const GroupedGemm &g, hipStream_t s) {
  hipLaunchKernelGGL((ggemm_dma_kernel<BM, BN, WGM, WGN>), dim3(g.total_tiles),
                     dim3(64 * WGM * WGN), 0, s, g);
}


template <int BM, int BN, int BK, int WGM, int WGN, int PREC>
void launch_tile(const GemmDesc &g, hipStream_t s) {
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  dim3 grid(tiles), block(64 * WGM * WGN);
  if (g.kfast_a && g.nfast_b)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WGM, WGN, true, true, PREC>), grid, block, 0, s,
                       g);
  else if (g.kfast_a)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WGM, WGN, true, false, PREC>), grid, block, 0, s,
                       g);
  else if (g.nfast_b)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WGM, WGN, false, true, PREC>), grid, block, 0, s,
                       g);
  else
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WGM, WGN, false, false, PREC>), grid, block, 0,
                       s, g);
  GXY_CHECK_LAUNCH();
}

template <int PREC>
void launch_tile_prec(const GemmDesc &g, hipStream_t s) {
  constexpr int BK = PREC == kB3 ? 32 : 16;
  const int64_t big = (int64_t)((g.M + 127) / 128) * ((g.N + 127) / 128);
  if (g.K > 0 && big >= 512)
    launch_tile<128, 128, BK, 4, 2, PREC>(g, s);
  else
    launch_tile<64, 64, BK, 2, 2, PREC>(g, s);
}

template <int BM, int BN, int BK, int WGM, int WGN, int PREC>
void launch_grouped(const GroupedGemm &g, hipStream_t s) {
  if (g.sym && (BM != BN || g.contig || g.beta != 0.0))
    fail(GXY_EDEVICE, "symmetric grouped GEMM: square tiles, table addressing, beta = 0");
  dim3 grid(g.total_tiles), block(64 * WGM * WGN);
  if (g.contig) {
    bool dma = false;
    if constexpr (PREC == kF64) dma = g.dma;
    if (dma)
      launch_dma<BM, BN, WGM, WGN>(g, s);
    else
      hipLaunchKernelGGL((ggemm_contig_kernel<BM, BN, BK, WGM, WGN, PREC>), grid, block, 0, s, g);
  } else if (g.kfast_a && g.nfast_b)
    hipLaunchKernelGGL((ggemm_kernel<BM, BN, BK, WGM, WGN, true, true, PREC>), grid, block, 0, s,
                       g);
  else if (g.kfast_a)
    hipLaunchKernelGGL((ggemm_kernel<BM, BN, BK, WGM, WGN, true, false, PREC>), grid, block, 0,
                       s, g);
  else if (g.nfast_b)
    hipLaunchKernelGGL((ggemm_kernel<BM, BN, BK, WGM, WGN, false, true, PREC>), grid, block, 0,
                       s, g);
  else
    hipLaunchKernelGGL((ggemm_kernel<BM, BN, BK, WGM, WGN, false, false, PREC>), grid, block, 0,
                       s, g);
  GXY_CHECK_LAUNCH();
}

template <int PREC>
void launch_grouped_prec(const GroupedGemm &g, hipStream_t s) {
  // k-slice depth: 8 for FP64 (the D = 64 projection product alone, 128 x
  // 128 tile: 45.5 against 40.9 TF/s with 16; same accumulation order, so
  // the same bits), 16 for FP32, 32 for BF16x3 (one 16x16x32 step)
  constexpr int BK = PREC == kB3 ? 32 : (PREC == kF64 ? 8 : 16);
  if (g.tile == 256)
    launch_grouped<256, 128, BK, 4, 2, PREC>(g, s);
  else if (g.tile == 128)
    launch_grouped<128, 128, BK, 4, 2, PREC>(g, s);
  else
    launch_grouped<64, 64, BK, 2, 2, PREC>(g, s);
}

// One wave: lane l supplies a[l], b[l]; out[4 l + r] = result register r.
__global__ void mfma_probe_kernel(const double *a, const double *b, double *out) {
  const int l = threadIdx.x;
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[l], b[l], acc, 0, 0, 0);
  for (int r = 0; r < 4; ++r) out[4 * l + r] = acc[r];
}

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// kind 0: v_mfma_f32_16x16x4_f32 with a[l], b[l];
// kind 1: v_mfma_f32_16x16x32_bf16 with a[8 l + j], b[8 l + j] (j < 8) as bf16.
__global__ void mfma_probe32_kernel(int kind, const float *a, const float *b, float *out) {
  const int l = threadIdx.x;
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
  if (kind == 0) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[l], b[l], acc, 0, 0, 0);
  } else {
    bf16x8_t av, bv;
    for (int j = 0; j < 8; ++j) {
      av[j] = (__bf16)a[8 * l + j];
      bv[j] = (__bf16)b[8 * l + j];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
  for (int r = 0; r < 4; ++r) out[4 * l + r] = acc[r];
}

}  // namespace

void launch_mfma_probe32(int kind, const float *a, const float *b, float *out,
                         hipStream_t s) {
  hipLaunchKernelGGL(mfma_probe32_kernel, dim3(1), dim3(64), 0, s, kind, a, b, out);
  GXY_CHECK_LAUNCH();
}

void gemm(const GemmDesc &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return;
  switch (g.prec) {
    case kF64: launch_tile_prec<kF64>(g, s); break;
    case kF32: launch_tile_prec<kF32>(g, s); break;
    case kB3: launch_tile_prec<kB3>(g, s); break;
    default: fail(GXY_EUNSUPPORTED, "GEMM: unknown precision");
  }
}

void grouped_gemm(const GroupedGemm &g, hipStream_t s) {
  if (g.ngroups <= 0 || g.total_tiles <= 0) return;
  switch (g.prec) {
    case kF64: launch_grouped_prec<kF64>(g, s); break;
    case kF32: launch_grouped_prec<kF32>(g, s); break;
    case kB3: launch_grouped_prec<kB3>(g, s); break;
    default: fail(GXY_EUNSUPPORTED, "grouped GEMM: unknown precision");
  }
}

void launch_mfma_probe(const double *a, const double *b, double *out, hipStream_t s) {
  hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, s, a, b, out);
  GXY_CHECK_LAUNCH();
}

}  // namespace gxy
