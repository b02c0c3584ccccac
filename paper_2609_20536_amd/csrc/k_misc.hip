// Norms, scalings, leg permutations, traces, truncation/selection, projector
// assembly and the final log-norm accumulation (all FP64).
#include "internal.h"

#include <float.h>

namespace gxy {

namespace {

constexpr int kRedThreads = 256;
constexpr int kNormBlocks = 1024;

template <int NT>
__device__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__global__ void sumsq_partial_kernel(const double *x, int64_t n, double *partial) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kRedThreads;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride)
    acc += x[i] * x[i];
  double s = block_sum<kRedThreads>(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void norm_final_kernel(const double *partial, int nb, double *out3) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kRedThreads) acc += partial[i];
  double s = block_sum<kRedThreads>(acc, red);
  if (threadIdx.x == 0) {
    const double c = sqrt(s);
    out3[0] = c;
    out3[1] = log(c);
    out3[2] = 1.0 / c;
  }
}

__global__ void scale_kernel(double *x, int64_t n, const double *scale) {
  const double c = *scale;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    x[i] *= c;
}

// out[j][i] = in[i][j] for an R x C matrix (tiled through LDS).
__global__ void transpose_kernel(const double *in, double *out, int64_t R, int64_t C) {
  __shared__ double tile[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    if (r < R && c < C) tile[k][tx] = in[r * C + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (r < R && c < C) out[c * R + r] = tile[tx][k];
  }
}

__global__ void swap_middle_kernel(const double *in, double *out, int A, int B,
                                   int C, int D) {
  const int64_t total = (int64_t)A * B * C * D;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int d = (int)(e % D);
    int64_t t = e / D;
    const int b = (int)(t % B);
    t /= B;
    const int c = (int)(t % C);
    const int a = (int)(t / C);
    // out[a][c][b][d] = in[a][b][c][d]; e enumerates out in order (a, c, b, d)
    out[e] = in[(((int64_t)a * B + b) * C + c) * D + d];
  }
}

// out[P1 * W + P2] = in[l][r][u][d] with (l, u) = pinv[P1], (r, d) = pinv[P2]
// (pinv[P] = h * Dv + v, W = Dh * Dv): the bottom operand of the D^7 product
// with both fused indices in block order.
__global__ void block_gather_kernel(const double *in, double *out, const int32_t *pinv, int Dh,
                                    int Dv) {
  const int64_t W = (int64_t)Dh * Dv, total = W * W;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int f1 = pinv[e / W], f2 = pinv[e % W];
    const int l = f1 / Dv, u = f1 % Dv, r = f2 / Dv, d = f2 % Dv;
    out[e] = in[(((int64_t)l * Dh + r) * Dv + u) * Dv + d];
  }
}

__global__ void trace_kernel(const double *T, int Dh, int Dv, double *out) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  const int64_t n = (int64_t)Dh * Dv;
  for (int64_t i = threadIdx.x; i < n; i += kRedThreads) {
    const int l = (int)(i / Dv), u = (int)(i % Dv);
    acc += T[(((int64_t)l * Dh + l) * Dv + u) * Dv + u];
  }
  double s = block_sum<kRedThreads>(acc, red);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ void fill_kernel(double *x, int64_t n, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    x[i] = v;
}

__global__ void fill_i32_kernel(int32_t *x, int64_t n, int32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    x[i] = v;
}

__global__ void identity_kernel(double *P, int n) {
  const int64_t total = (int64_t)n * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
    P[i] = (i / n == i % n) ? 1.0 : 0.0;
}

unsigned grid_for(int64_t n, int per = 256, unsigned cap = 8192) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ---------------------------------------------------------------------------
// Truncation (Ch. 2, HOTRG: keep the leading Dcut mode vectors of the side
// with the smaller discarded weight). One block per side finds the kept
// states with the tie rule; a second kernel chooses the side.
// ---------------------------------------------------------------------------

constexpr int kSelThreads = 1024;

__device__ double block_max(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = kSelThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_min(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = kSelThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__device__ unsigned long long block_min_u64(unsigned long long v, unsigned long long *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = kSelThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      unsigned long long o = red[threadIdx.x + off];
      if (o < red[threadIdx.x]) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  unsigned long long r = red[0];
  __syncthreads();
  return r;
}

__device__ int block_sum_i(int v, int *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = kSelThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  int r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_sum_d(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = kSelThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__device__ unsigned long long tie_key(int label, int rank) {
  const unsigned long long aq = (unsigned long long)(label < 0 ? -label : label);
  const unsigned long long sq = (unsigned long long)(label + 32768);
  return (aq << 40) | (sq << 24) | (unsigned long long)rank;
}

// per side: writes side_res[side*8 + {0 eps, 1 trE, 2 lam1, 3 gap, 4 ties}],
// side_pick_{sec,col,rank}[side*dcut + p]. General form for any number of
// candidates: they stay in global memory.
__global__ void select_side_wide_kernel(SelectArgs a, double *side_res,
                                   int32_t *side_pick_sec, int32_t *side_pick_col,
                                   int32_t *side_pick_rank) {
  __shared__ double redd[kSelThreads];
  __shared__ unsigned long long redu[kSelThreads];
  __shared__ int redi[kSelThreads];
  __shared__ int sec_start_s[1];
  const int side = blockIdx.x;
  const int nsec = a.nsec;
  const int nc = a.ncand;
  double *lam = a.d_lam + (int64_t)side * nc;
  int32_t *csec = a.d_cand_sec + (int64_t)side * nc;
  int32_t *crank = a.d_cand_rank + (int64_t)side * nc;
  int32_t *ccol = a.d_cand_col + (int64_t)side * nc;
  int32_t *taken = a.d_taken + (int64_t)side * nc;
  (void)sec_start_s;

  // 1. candidates: eigenvalue = diagonal of the converged padded matrix
  int base = 0;
  for (int s = 0; s < nsec; ++s) {
    const int n = a.d_sec_n[s];
    const int mi = side * nsec + s;
    const double *Am = a.A + a.d_mat_off[mi];
    const int npad = a.d_mat_npad[mi];
    for (int i = threadIdx.x; i < n; i += kSelThreads) {
      lam[base + i] = Am[(int64_t)i * npad + i];
      csec[base + i] = s;
      ccol[base + i] = i;
      taken[base + i] = 0;
    }
    base += n;
  }
  __syncthreads();
  // within-sector rank by decreasing eigenvalue (ties by column)
  base = 0;
  for (int s = 0; s < nsec; ++s) {
    const int n = a.d_sec_n[s];
    for (int i = threadIdx.x; i < n; i += kSelThreads) {
      const double li = lam[base + i];
      int r = 0;
      for (int j = 0; j < n; ++j) {
        const double lj = lam[base + j];
        r += (lj > li || (lj == li && j < i)) ? 1 : 0;
      }
      crank[base + i] = r;
    }
    base += n;
  }
  __syncthreads();

  // 2. greedy picks with the tie rule
  double lam1 = -DBL_MAX;
  int ties = 0, bad = 0;
  for (int p = 0; p < a.dcut; ++p) {
    double v = -DBL_MAX;
    for (int c = threadIdx.x; c < nc; c += kSelThreads)
      if (!taken[c]) v = fmax(v, lam[c]);
    const double top = block_max(v, redd);
    if (p == 0) lam1 = top;
    const double tol = a.tie_rel * fabs(lam1);
    unsigned long long kbest = ~0ull;
    int cnt = 0;
    for (int c = threadIdx.x; c < nc; c += kSelThreads) {
      if (!taken[c] && lam[c] >= top - tol) {
        ++cnt;
        const unsigned long long k = tie_key(a.d_sec_label[csec[c]], crank[c]);
        if (k < kbest) kbest = k;
      }
    }
    kbest = block_min_u64(kbest, redu);
    cnt = block_sum_i(cnt, redi);
    if (cnt > 1) ++ties;
    if (cnt == 0) {
      // no finite candidate left (a non-finite spectrum): a valid state
      // stands in and the side's lambda_1 becomes NaN for the host to see
      bad = 1;
      if (threadIdx.x == 0) {
        side_pick_sec[side * a.dcut + p] = 0;
        side_pick_col[side * a.dcut + p] = 0;
        side_pick_rank[side * a.dcut + p] = 0;
      }
    }
    for (int c = threadIdx.x; c < nc; c += kSelThreads) {
      if (!taken[c] && lam[c] >= top - tol &&
          tie_key(a.d_sec_label[csec[c]], crank[c]) == kbest) {
        taken[c] = 1;
        side_pick_sec[side * a.dcut + p] = csec[c];
        side_pick_col[side * a.dcut + p] = ccol[c];
        side_pick_rank[side * a.dcut + p] = crank[c];
      }
    }
    __syncthreads();
  }

  // 3. discarded weight, trace, cut gap (fixed-order reductions)
  double eps = 0.0, tr = 0.0, minkept = DBL_MAX, maxdisc = -DBL_MAX;
  for (int c = threadIdx.x; c < nc; c += kSelThreads) {
    tr += lam[c];
    if (taken[c]) {
      minkept = fmin(minkept, lam[c]);
    } else {
      eps += lam[c];
      maxdisc = fmax(maxdisc, lam[c]);
    }
  }
  eps = block_sum_d(eps, redd);
  tr = block_sum_d(tr, redd);
  minkept = block_min(minkept, redd);
  maxdisc = block_max(maxdisc, redd);
  if (threadIdx.x == 0) {
    side_res[side * 8 + 0] = eps;
    side_res[side * 8 + 1] = tr;
    side_res[side * 8 + 2] = bad ? NAN : lam1;
    side_res[side * 8 + 3] = lam1 > 0.0 ? (minkept - maxdisc) / lam1 : 0.0;
    side_res[side * 8 + 4] = (double)ties;
  }
}


// The same selection with each thread's candidates (c = thread + k
// kSelThreads) held in registers, for at most kSelThreads kSelPer candidates
// per side: the greedy picks then touch no global memory, and their
// reductions are one wave-level pass plus one barrier each. Maximum, minimum
// and counts are exact in any order, and the discarded weight and trace are
// summed in the order of the general form, so both give the same bits. A
// sector whose eigenvalues arrive in non-increasing order (the tridiagonal
// path's) has rank = column; any other sector is ranked by comparisons.
constexpr int kSelPer = 12;
constexpr int kSelWaves = kSelThreads / 64;

__device__ __forceinline__ double sel_wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__global__ __launch_bounds__(kSelThreads) void select_side_kernel(
    SelectArgs a, double *side_res, int32_t *side_pick_sec, int32_t *side_pick_col,
    int32_t *side_pick_rank) {
  __shared__ double redd[kSelThreads];
  __shared__ double wmax[2][kSelWaves];
  __shared__ unsigned long long wkey[kSelWaves];
  __shared__ int wcnt[kSelWaves];
  __shared__ int unsorted;
  const int side = blockIdx.x;
  const int nsec = a.nsec;
  const int nc = a.ncand;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *lam = a.d_lam + (int64_t)side * nc;
  int32_t *csec = a.d_cand_sec + (int64_t)side * nc;
  int32_t *crank = a.d_cand_rank + (int64_t)side * nc;
  int32_t *ccol = a.d_cand_col + (int64_t)side * nc;
  if (tid == 0) unsorted = 0;

  // 1. candidates: eigenvalue = diagonal of the converged padded matrix
  int base = 0;
  for (int s = 0; s < nsec; ++s) {
    const int n = a.d_sec_n[s];
    const int mi = side * nsec + s;
    const double *Am = a.A + a.d_mat_off[mi];
    const int npad = a.d_mat_npad[mi];
    for (int i = tid; i < n; i += kSelThreads) {
      lam[base + i] = Am[(int64_t)i * npad + i];
      csec[base + i] = s;
      ccol[base + i] = i;
      crank[base + i] = i;
    }
    base += n;
  }
  __syncthreads();
  for (int c = tid; c + 1 < nc; c += kSelThreads)
    if (csec[c] == csec[c + 1] && lam[c] < lam[c + 1]) unsorted = 1;
  __syncthreads();
  if (unsorted) {
    // within-sector rank by decreasing eigenvalue (ties by column)
    base = 0;
    for (int s = 0; s < nsec; ++s) {
      const int n = a.d_sec_n[s];
      for (int i = tid; i < n; i += kSelThreads) {
        const double li = lam[base + i];
        int r = 0;
        for (int j = 0; j < n; ++j) {
          const double lj = lam[base + j];
          r += (lj > li || (lj == li && j < i)) ? 1 : 0;
        }
        crank[base + i] = r;
      }
      base += n;
    }
    __syncthreads();
  }
  double rl[kSelPer];
  unsigned long long rk[kSelPer];
  unsigned out = 0;   // bit k: candidate k taken (or absent)
#pragma unroll
  for (int k = 0; k < kSelPer; ++k) {
    const int c = tid + k * kSelThreads;
    if (c < nc) {
      rl[k] = lam[c];
      rk[k] = tie_key(a.d_sec_label[csec[c]], crank[c]);
    } else {
      rl[k] = -DBL_MAX;
      rk[k] = ~0ull;
      out |= 1u << k;
    }
  }

  // 2. greedy picks with the tie rule
  double lam1 = -DBL_MAX;
  int ties = 0, bad = 0;
  for (int p = 0; p < a.dcut; ++p) {
    double v = -DBL_MAX;
#pragma unroll
    for (int k = 0; k < kSelPer; ++k)
      if (!((out >> k) & 1u)) v = fmax(v, rl[k]);
    v = sel_wave_max(v);
    if (lane == 0) wmax[p & 1][wave] = v;
    __syncthreads();
    double top = wmax[p & 1][0];
    for (int w = 1; w < kSelWaves; ++w) top = fmax(top, wmax[p & 1][w]);
    if (p == 0) lam1 = top;
    const double tol = a.tie_rel * fabs(lam1);
    unsigned long long kbest = ~0ull;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < kSelPer; ++k)
      if (!((out >> k) & 1u) && rl[k] >= top - tol) {
        ++cnt;
        if (rk[k] < kbest) kbest = rk[k];
      }
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long ko = __shfl_xor(kbest, o, 64);
      if (ko < kbest) kbest = ko;
      cnt += __shfl_xor(cnt, o, 64);
    }
    if (lane == 0) {
      wkey[wave] = kbest;
      wcnt[wave] = cnt;
    }
    __syncthreads();
    kbest = wkey[0];
    cnt = wcnt[0];
    for (int w = 1; w < kSelWaves; ++w) {
      if (wkey[w] < kbest) kbest = wkey[w];
      cnt += wcnt[w];
    }
    if (cnt > 1) ++ties;
    if (cnt == 0) {
      // no finite candidate left (a non-finite spectrum): a valid state
      // stands in and the side's lambda_1 becomes NaN for the host to see
      bad = 1;
      if (tid == 0) {
        side_pick_sec[side * a.dcut + p] = 0;
        side_pick_col[side * a.dcut + p] = 0;
        side_pick_rank[side * a.dcut + p] = 0;
      }
    }
    int kw = -1;   // the one candidate with the winning key, if this thread holds it
#pragma unroll
    for (int k = 0; k < kSelPer; ++k)
      if (!((out >> k) & 1u) && rl[k] >= top - tol && rk[k] == kbest) kw = k;
    if (kw >= 0) {
      const int c = tid + kw * kSelThreads;
      out |= 1u << kw;
      side_pick_sec[side * a.dcut + p] = csec[c];
      side_pick_col[side * a.dcut + p] = ccol[c];
      side_pick_rank[side * a.dcut + p] = crank[c];
    }
    // (no barrier needed here: the next pick writes the other wmax buffer,
    // and wkey only after its first barrier, which every thread reaches
    // after reading this pick's wkey)
  }

  // 3. discarded weight, trace, cut gap (fixed-order reductions)
  double eps = 0.0, tr = 0.0, minkept = DBL_MAX, maxdisc = -DBL_MAX;
#pragma unroll
  for (int k = 0; k < kSelPer; ++k) {
    if (tid + k * kSelThreads >= nc) continue;
    tr += rl[k];
    if ((out >> k) & 1u) {
      minkept = fmin(minkept, rl[k]);
    } else {
      eps += rl[k];
      maxdisc = fmax(maxdisc, rl[k]);
    }
  }
  eps = block_sum_d(eps, redd);
  tr = block_sum_d(tr, redd);
  minkept = block_min(minkept, redd);
  maxdisc = block_max(maxdisc, redd);
  if (tid == 0) {
    side_res[side * 8 + 0] = eps;
    side_res[side * 8 + 1] = tr;
    side_res[side * 8 + 2] = bad ? NAN : lam1;
    side_res[side * 8 + 3] = lam1 > 0.0 ? (minkept - maxdisc) / lam1 : 0.0;
    side_res[side * 8 + 4] = (double)ties;
  }
}

__global__ void select_final_kernel(SelectArgs a, const double *side_res,
                                    const int32_t *side_pick_sec,
                                    const int32_t *side_pick_col,
                                    const int32_t *side_pick_rank) {
  const double epsL = side_res[0], epsR = side_res[8];
  // (a NaN lambda_1 marks a side without enough finite states: kept)
  const double lmax = (isnan(side_res[2]) || isnan(side_res[10])) ? NAN
                                                                   : fmax(side_res[2], side_res[10]);
  const int side = (epsR < epsL - a.side_tol * lmax) ? 1 : 0;
  const int D = a.dcut;
  const int32_t *ps = side_pick_sec + side * D;
  const int32_t *pc = side_pick_col + side * D;
  const int32_t *pr = side_pick_rank + side * D;
  // order the kept states by (label, rank)
  for (int p = threadIdx.x; p < D; p += blockDim.x) {
    const long long kp = (long long)a.d_sec_label[ps[p]] * (1ll << 32) + pr[p];
    int pos = 0;
    for (int q = 0; q < D; ++q) {
      const long long kq = (long long)a.d_sec_label[ps[q]] * (1ll << 32) + pr[q];
      pos += (kq < kp) ? 1 : 0;
    }
    a.d_pick_sec[pos] = ps[p];
    a.d_pick_col[pos] = pc[p];
    a.d_pick_label[pos] = a.d_sec_label[ps[p]];
  }
  if (threadIdx.x == 0) {
    a.d_diag[0] = epsL;
    a.d_diag[1] = epsR;
    a.d_diag[2] = (double)side;
    a.d_diag[3] = lmax;
    a.d_diag[4] = side_res[side * 8 + 3];
    a.d_diag[5] = side_res[side * 8 + 4];
    a.d_diag[6] = side_res[side * 8 + 1];
  }
}

__global__ void build_projector_kernel(const double *V, const int64_t *mat_off,
                                       const int32_t *mat_npad,
                                       const int32_t *sec_idx,
                                       const int32_t *sec_start,
                                       const int32_t *sec_n,
                                       const int32_t *pick_sec,
                                       const int32_t *pick_col,
                                       const double *diag, int nsec, int dcut,
                                       double *P) {
  const int j = blockIdx.x;
  const int side = (int)diag[2];
  const int s = pick_sec[j];
  const int col = pick_col[j];
  const int mi = side * nsec + s;
  const double *Vm = V + mat_off[mi];
  const int npad = mat_npad[mi];
  const int n = sec_n[s];
  const int st = sec_start[s];
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    P[(int64_t)sec_idx[st + i] * dcut + j] = Vm[(int64_t)i * npad + col];
}

struct TraceSet {
  const double *t[4];   // cos, cos q, cos^2, cos^2 q (null if not carried)
};

__global__ void finish_kernel(const double *lnc, int nsteps, double beta, const double *tr,
                              TraceSet tk, double *res) {
  if (threadIdx.x != 0) return;
  double acc = lnc[0];
  for (int n = 1; n <= nsteps; ++n) acc += lnc[n] / ldexp(1.0, n);
  const double t = tr[0];
  const bool ok = (t > 0.0) && isfinite(t) && isfinite(acc);
  res[0] = ok ? acc + log(t) / ldexp(1.0, nsteps) : NAN;
  res[1] = tk.t[0] ? tk.t[0][0] / t : NAN;
  res[2] = tk.t[1] ? tk.t[1][0] / t : NAN;
  res[3] = ok ? 0.0 : (double)GXY_ENUMERIC;
  // second moments of the site averages and beta V (<m^2> - <m>^2)
  const double V = ldexp(1.0, nsteps);
  for (int j = 0; j < 2; ++j) {
    const double msq = tk.t[2 + j] ? tk.t[2 + j][0] / t : NAN;
    res[4 + j] = msq;
    res[6 + j] = beta * V * (msq - res[1 + j] * res[1 + j]);
  }
}

__global__ void observables_kernel(int npts, const double *beta, const double *lnz,
                                   const double *mh, const double *mh1,
                                   double dbeta, double dh, double dh1, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  const double b = beta[i];
  const double *l = lnz + 3 * i;
  out[4 * i + 0] = -l[1] / b;
  out[4 * i + 1] = b * b * (l[2] - 2.0 * l[1] + l[0]) / (dbeta * dbeta);
  out[4 * i + 2] = (mh[2 * i + 1] - mh[2 * i]) / (2.0 * dh);
  out[4 * i + 3] = (mh1[2 * i + 1] - mh1[2 * i]) / (2.0 * dh1);
}

}  // namespace

void launch_fro_norm(const double *x, int64_t n, double *partial, double *out3,
                     hipStream_t s) {
  hipLaunchKernelGGL(sumsq_partial_kernel, dim3(kNormBlocks), dim3(kRedThreads), 0,
                     s, x, n, partial);
  GXY_CHECK_LAUNCH();
  hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(kRedThreads), 0, s, partial,
                     kNormBlocks, out3);
  GXY_CHECK_LAUNCH();
}

void launch_scale(double *x, int64_t n, const double *scale, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, scale);
  GXY_CHECK_LAUNCH();
}

void launch_swap_pairs(const double *in, double *out, int A, int B, int C, int D,
                       hipStream_t s) {
  const int64_t R = (int64_t)A * B, Cc = (int64_t)C * D;
  dim3 grid((unsigned)((Cc + 31) / 32), (unsigned)((R + 31) / 32));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, in, out, R, Cc);
  GXY_CHECK_LAUNCH();
}

void launch_swap_middle(const double *in, double *out, int A, int B, int C, int D,
                        hipStream_t s) {
  const int64_t n = (int64_t)A * B * C * D;
  hipLaunchKernelGGL(swap_middle_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out,
                     A, B, C, D);
  GXY_CHECK_LAUNCH();
}

void launch_block_gather(const double *in, double *out, const int32_t *pinv, int Dh, int Dv,
                         hipStream_t s) {
  const int64_t n = (int64_t)Dh * Dv * Dh * Dv;
  hipLaunchKernelGGL(block_gather_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, pinv, Dh,
                     Dv);
  GXY_CHECK_LAUNCH();
}

void launch_trace(const double *T, int Dh, int Dv, double *out, hipStream_t s) {
  hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(kRedThreads), 0, s, T, Dh, Dv, out);
  GXY_CHECK_LAUNCH();
}

void launch_fill(double *x, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, v);
  GXY_CHECK_LAUNCH();
}

void launch_fill_i32(int32_t *x, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, v);
  GXY_CHECK_LAUNCH();
}

void launch_identity(double *P, int n, hipStream_t s) {
  hipLaunchKernelGGL(identity_kernel, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s,
                     P, n);
  GXY_CHECK_LAUNCH();
}

void launch_select(const SelectArgs &a, hipStream_t s) {
  // side results and per-side picks live after the candidate arrays
  double *side_res = a.d_diag + 8;                  // 16 doubles
  int32_t *sps = a.d_taken + 2 * (int64_t)a.ncand;  // 3 * 2 * dcut ints
  int32_t *spc = sps + 2 * a.dcut;
  int32_t *spr = spc + 2 * a.dcut;
  if (a.ncand <= kSelThreads * kSelPer)
    hipLaunchKernelGGL(select_side_kernel, dim3(2), dim3(kSelThreads), 0, s, a, side_res,
                       sps, spc, spr);
  else
    hipLaunchKernelGGL(select_side_wide_kernel, dim3(2), dim3(kSelThreads), 0, s, a,
                       side_res, sps, spc, spr);
  GXY_CHECK_LAUNCH();
  hipLaunchKernelGGL(select_final_kernel, dim3(1), dim3(256), 0, s, a, side_res, sps,
                     spc, spr);
  GXY_CHECK_LAUNCH();
}

void launch_build_projector(const double *V, const int64_t *d_mat_off,
                            const int32_t *d_mat_npad, const int32_t *d_sec_idx,
                            const int32_t *d_sec_start, const int32_t *d_sec_n,
                            const int32_t *d_pick_sec, const int32_t *d_pick_col,
                            const double *d_diag, int nsec, int nfused, int dcut,
                            double *P, hipStream_t s) {
  launch_fill(P, (int64_t)nfused * dcut, 0.0, s);
  hipLaunchKernelGGL(build_projector_kernel, dim3(dcut), dim3(256), 0, s, V, d_mat_off,
                     d_mat_npad, d_sec_idx, d_sec_start, d_sec_n, d_pick_sec,
                     d_pick_col, d_diag, nsec, dcut, P);
  GXY_CHECK_LAUNCH();
}

void launch_finish(const double *lnc, int nsteps, double beta, const double *tr,
                   const double *const trk[4], double *res, hipStream_t s) {
  TraceSet tk{{trk[0], trk[1], trk[2], trk[3]}};
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, lnc, nsteps, beta, tr, tk, res);
  GXY_CHECK_LAUNCH();
}

void launch_observables(int npts, const double *beta, const double *lnz,
                        const double *mh, const double *mh1, double dbeta,
                        double dh, double dh1, double *out, hipStream_t s) {
  hipLaunchKernelGGL(observables_kernel, dim3((npts + 63) / 64), dim3(64), 0, s, npts,
                     beta, lnz, mh, mh1, dbeta, dh, dh1, out);
  GXY_CHECK_LAUNCH();
}

}  // namespace gxy
