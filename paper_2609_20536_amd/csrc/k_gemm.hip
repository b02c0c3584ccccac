// FP64 MFMA GEMMs with index-fused operands for the HOTRG contractions.
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
// Tiling for CDNA4: 256 threads = 4 wave64s in a 2x2 arrangement; each wave
// owns a (BM/2) x (BN/2) sub-tile made of 16x16 blocks computed with
// v_mfma_f64_16x16x4_f64. A and B tiles (BK = 16) are staged through LDS with
// the next tile's global loads in flight while the current one is consumed.
// Workgroups are renumbered so that each XCD (own L2) works on a contiguous
// band of output tiles.
#include "internal.h"

namespace gxy {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kBK = 16;

struct AffineAddr {
  const IdxMap *am, *ak, *bk, *bn, *cm, *cn;
  __device__ int64_t a_m(int m) const { return imap_off(*am, m); }
  __device__ int64_t a_k(int k) const { return imap_off(*ak, k); }
  __device__ int64_t b_k(int k) const { return imap_off(*bk, k); }
  __device__ int64_t b_n(int n) const { return imap_off(*bn, n); }
  __device__ int64_t c_m(int m) const { return imap_off(*cm, m); }
  __device__ int64_t c_n(int n) const { return imap_off(*cn, n); }
};

struct TableAddr {
  const int64_t *ar, *ac, *br, *bc, *cr, *cc;
  __device__ int64_t a_m(int m) const { return ar[m]; }
  __device__ int64_t a_k(int k) const { return ac[k]; }
  __device__ int64_t b_k(int k) const { return br[k]; }
  __device__ int64_t b_n(int n) const { return bc[n]; }
  __device__ int64_t c_m(int m) const { return cr[m]; }
  __device__ int64_t c_n(int n) const { return cc[n]; }
};

// One BM x BN output tile of C(m, n) = alpha sum_k A(m, k) B(k, n) + beta C.
template <int BM, int BN, bool KFA, bool NFB, class Addr>
__device__ __forceinline__ void gemm_tile(const Addr &ad, int M, int N, int K, int m0, int n0,
                                          const double *__restrict__ A,
                                          const double *__restrict__ B, double *C,
                                          double alpha, double beta,
                                          double (*As)[BM + 1], double (*Bs)[BN + 1]) {
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_PER = BM * kBK / kThreads;
  constexpr int B_PER = BN * kBK / kThreads;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM;
  const int wn0 = (wave & 1) * WN;

  int64_t a_fixed[KFA ? A_PER : 1];
  bool a_ok[KFA ? A_PER : 1];
  if (KFA) {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      const int m = m0 + tid / kBK + 16 * p;
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
      const int n = n0 + tid / kBK + 16 * p;
      b_ok[p] = n < N;
      b_fixed[p] = b_ok[p] ? ad.b_n(n) : 0;
    }
  }

  double ra[A_PER], rb[B_PER];
  auto load_tiles = [&](int k0) {
    if (KFA) {
      const int k = k0 + tid % kBK;
      const bool kok = k < K;
      const int64_t ko = kok ? ad.a_k(k) : 0;
#pragma unroll
      for (int p = 0; p < A_PER; ++p) ra[p] = (kok && a_ok[p]) ? A[a_fixed[p] + ko] : 0.0;
    } else {
      constexpr int KSTEP = kThreads / BM;
#pragma unroll
      for (int p = 0; p < A_PER; ++p) {
        const int k = k0 + tid / BM + KSTEP * p;
        ra[p] = (k < K && a_ok[0]) ? A[a_fixed[0] + ad.a_k(k)] : 0.0;
      }
    }
    if (NFB) {
      constexpr int KSTEP = kThreads / BN;
#pragma unroll
      for (int p = 0; p < B_PER; ++p) {
        const int k = k0 + tid / BN + KSTEP * p;
        rb[p] = (k < K && b_ok[0]) ? B[ad.b_k(k) + b_fixed[0]] : 0.0;
      }
    } else {
      const int k = k0 + tid % kBK;
      const bool kok = k < K;
      const int64_t ko = kok ? ad.b_k(k) : 0;
#pragma unroll
      for (int p = 0; p < B_PER; ++p) rb[p] = (kok && b_ok[p]) ? B[ko + b_fixed[p]] : 0.0;
    }
  };
  auto store_tiles = [&]() {
    if (KFA) {
#pragma unroll
      for (int p = 0; p < A_PER; ++p) As[tid % kBK][tid / kBK + 16 * p] = ra[p];
    } else {
      constexpr int KSTEP = kThreads / BM;
#pragma unroll
      for (int p = 0; p < A_PER; ++p) As[tid / BM + KSTEP * p][tid % BM] = ra[p];
    }
    if (NFB) {
      constexpr int KSTEP = kThreads / BN;
#pragma unroll
      for (int p = 0; p < B_PER; ++p) Bs[tid / BN + KSTEP * p][tid % BN] = rb[p];
    } else {
#pragma unroll
      for (int p = 0; p < B_PER; ++p) Bs[tid % kBK][tid / kBK + 16 * p] = rb[p];
    }
  };

  double4_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

  const int ktiles = (K + kBK - 1) / kBK;
  if (ktiles > 0) load_tiles(0);
  for (int kt = 0; kt < ktiles; ++kt) {
    store_tiles();
    __syncthreads();
    if (kt + 1 < ktiles) load_tiles((kt + 1) * kBK);
    const int li = lane & 15;
    const int lk = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      double fa[FM], fb[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) fa[i] = As[kk + lk][wm0 + 16 * i + li];
#pragma unroll
      for (int j = 0; j < FN; ++j) fb[j] = Bs[kk + lk][wn0 + 16 * j + li];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  // the f64 16x16x4 accumulator of lane l holds rows l/16 + 4r (r = 0..3) of
  // column l%16
  const int cr = lane >> 4;
  const int cc = lane & 15;
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int n = n0 + wn0 + 16 * j + cc;
    if (n >= N) continue;
    const int64_t noff = ad.c_n(n);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm0 + 16 * i + cr + 4 * r;
        if (m >= M) continue;
        double *dst = C + ad.c_m(m) + noff;
        const double v = alpha * acc[i][j][r];
        *dst = (beta == 0.0) ? v : v + beta * (*dst);
      }
    }
  }
}

__device__ __forceinline__ int xcd_remap(int pid, int total) {
  return ((total & 7) == 0) ? (pid & 7) * (total >> 3) + (pid >> 3) : pid;
}

template <int BM, int BN, bool KFA, bool NFB>
__global__ __launch_bounds__(kThreads) void gemm_f64_kernel(GemmDesc g) {
  __shared__ double As[kBK][BM + 1];
  __shared__ double Bs[kBK][BN + 1];
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
  gemm_tile<BM, BN, KFA, NFB>(ad, g.M, g.N, g.K, tm * BM, tn * BN, g.A, g.B, g.C, g.alpha,
                              g.beta, As, Bs);
}

template <int BM, int BN, bool KFA, bool NFB>
__global__ __launch_bounds__(kThreads) void ggemm_f64_kernel(GroupedGemm g) {
  __shared__ double As[kBK][BM + 1];
  __shared__ double Bs[kBK][BN + 1];
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
  const int tm = local / tiles_n, tn = local % tiles_n;
  TableAddr ad{g.tab + G.ar, g.tab + G.ac, g.tab + G.br, g.tab + G.bc, g.tab + G.cr,
               g.tab + G.cc};
  gemm_tile<BM, BN, KFA, NFB>(ad, G.M, G.N, G.K, tm * BM, tn * BN, g.A, g.B, g.C, g.alpha,
                              g.beta, As, Bs);
}

template <int BM, int BN>
void launch_tile(const GemmDesc &g, hipStream_t s) {
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  dim3 grid(tiles), block(kThreads);
  if (g.kfast_a && g.nfast_b)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, true, true>), grid, block, 0, s, g);
  else if (g.kfast_a)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, true, false>), grid, block, 0, s, g);
  else if (g.nfast_b)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, false, true>), grid, block, 0, s, g);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, false, false>), grid, block, 0, s, g);
  GXY_CHECK_LAUNCH();
}

template <int BM, int BN>
void launch_grouped(const GroupedGemm &g, hipStream_t s) {
  dim3 grid(g.total_tiles), block(kThreads);
  if (g.kfast_a && g.nfast_b)
    hipLaunchKernelGGL((ggemm_f64_kernel<BM, BN, true, true>), grid, block, 0, s, g);
  else if (g.kfast_a)
    hipLaunchKernelGGL((ggemm_f64_kernel<BM, BN, true, false>), grid, block, 0, s, g);
  else if (g.nfast_b)
    hipLaunchKernelGGL((ggemm_f64_kernel<BM, BN, false, true>), grid, block, 0, s, g);
  else
    hipLaunchKernelGGL((ggemm_f64_kernel<BM, BN, false, false>), grid, block, 0, s, g);
  GXY_CHECK_LAUNCH();
}

// One wave: lane l supplies a[l], b[l]; out[4 l + r] = result register r.
__global__ void mfma_probe_kernel(const double *a, const double *b, double *out) {
  const int l = threadIdx.x;
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[l], b[l], acc, 0, 0, 0);
  for (int r = 0; r < 4; ++r) out[4 * l + r] = acc[r];
}

}  // namespace

void gemm_f64(const GemmDesc &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return;
  const int64_t big = (int64_t)((g.M + 127) / 128) * ((g.N + 127) / 128);
  if (g.K > 0 && big >= 512)
    launch_tile<128, 128>(g, s);
  else
    launch_tile<64, 64>(g, s);
}

void grouped_gemm_f64(const GroupedGemm &g, hipStream_t s) {
  if (g.ngroups <= 0 || g.total_tiles <= 0) return;
  if (g.tile == 128)
    launch_grouped<128, 128>(g, s);
  else
    launch_grouped<64, 64>(g, s);
}

void launch_mfma_probe(const double *a, const double *b, double *out, hipStream_t s) {
  hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, s, a, b, out);
  GXY_CHECK_LAUNCH();
}

}  // namespace gxy
