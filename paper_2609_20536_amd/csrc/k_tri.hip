// Batched FP64 symmetric eigensolver for sector matrices of up to 2048 rows:
// Householder tridiagonalisation, bisection for every eigenvalue, inverse
// iteration for the leading eigenvectors, back-transformation.
//
// The HOSVD factors of M (Ch. 2, eq. hosvd) are eigenvectors of the Gram
// matrices E of M's unfoldings, block diagonal in the symmetry label of the
// fused bond; every label sector of both sides is one matrix of the batch
// (gathered into padded row-major storage, row stride npad).
//
//  1. tri_reduce: one workgroup per matrix reduces A to tridiagonal form
//     T = H^T A H with n - 2 Householder reflectors, blocked: the reflectors
//     v and w-vectors of a panel of 16 columns are applied to the trailing
//     matrix together (a rank-32 update on the matrix cores, computed for
//     the tiles on and below the diagonal and written to both triangles, so
//     A stays exactly symmetric), and within the panel each column and each
//     matrix-vector product is corrected for the pending ones. Reflector j
//     is kept in row j of A (right of the diagonal). Sectors of at least
//     384 rows are shared by up to 8 workgroups of one cooperative launch
//     (a barrier of the matrix's workgroups per column).
//  2. tri_bisect: every eigenvalue of T by bisection on Sturm counts, a
//     group of 16 lanes each taking four halvings per round (all of them
//     enter the discarded weights).
//  3. tri_invit: the leading kq = min(n, Dcut) eigenvectors of T, one thread
//     per vector, by inverse iteration on the pivoted LU factorisation of
//     T - lambda I, then Gram-Schmidt across the workgroup (the textbook
//     bisection + inverse iteration pair for selected eigenpairs).
//  4. tri_back: the vectors are mapped back through the reflectors into V
//     (row-major, column c = c-th largest eigenvalue).
// Stages 1-2 (launch_tri_values) put the decreasing eigenvalues of every
// matrix on the diagonal of A for the selection; stages 3-4
// (launch_tri_vectors) can then be limited to the side the selection chose.
#include <float.h>
#include <stdlib.h>

#include <algorithm>

#include "internal.h"

namespace gxy {

namespace {

// 512 threads: the reduction's registers (up to 256 per lane at 8 waves per
// compute unit) then hold its working set without spilling; at 1024 threads
// (128 registers) about 90 values per lane spilled to scratch, whose reloads
// miss in the caches after every matrix-vector product has streamed A22
// through them (bench: 31.5 -> 39.7 steps/s).
constexpr int kRedThreads = 512;
constexpr int kRedWaves = kRedThreads / 64;

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// sum over the workgroup (every thread receives the total); red >= 16 slots
__device__ double block_sum(double x, double *red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kRedWaves; ++w) t += red[w];
  return t;
}

// Partial sums of A22 v over rows k in [k_lo, k_hi): acc[q] collects the
// elements lane + 64 q (q < Q = ceil(m / 64)). Loads past m read the last
// element of the row instead, so every lane loads unconditionally.
template <int Q>
__device__ __forceinline__ void mv_partial(const double *A22, int np, int m, int k_lo, int k_hi,
                                           const double *v, int lane, double *acc) {
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[q] = 0.0;
  int idx[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) idx[q] = min(lane + 64 * q, m - 1);
  for (int k = k_lo; k < k_hi; ++k) {
    const double vk = v[k];
    const double *ra = A22 + (int64_t)k * np;
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] += ra[idx[q]] * vk;
  }
}

// mv_partial<q> for q = nq (1 <= nq <= MAXN / 64), a chain of uniform tests
template <int MAXN, int Q = 1>
__device__ __forceinline__ void mv_dispatch(int nq, const double *A22, int np, int m, int k_lo,
                                            int k_hi, const double *v, int lane, double *acc) {
  if constexpr (Q <= MAXN / 64) {
    if (nq == Q) {
      mv_partial<Q>(A22, np, m, k_lo, k_hi, v, lane, acc);
      return;
    }
    mv_dispatch<MAXN, Q + 1>(nq, A22, np, m, k_lo, k_hi, v, lane, acc);
  }
}

// Panel width of the blocked reduction: the reflectors and w-vectors of kNb
// consecutive columns are applied to the trailing matrix together.
constexpr int kNb = 16;

// Sharing pays only for large sectors: every column costs a barrier of the
// matrix's workgroups, and they hold their compute units while they wait.
// Bench workload (largest sectors near 540 rows): 29.0 steps/s with the
// threshold at 512 rows, 29.9 at 384, 29.8 at 256, 28.9 at 768 (1024-thread
// workgroups); 39.9 at 384 and 39.7 at 256 with 512 threads.
constexpr int kMultiMinRows = 384;

// Workgroups that share one matrix in the multi-workgroup reduction: about
// 128 rows of A22 each, at most 8, and few enough that their private panels
// (2 kNb n values each) fit in the matrix's npad^2 scratch slot. Bench
// workload (largest sectors near 540 rows, 512-thread workgroups): 40.5
// steps/s with 128 rows per workgroup, 39.9 with 96, 40.3 with 192, 38.3
// with 64.
__host__ __device__ inline int tri_groups(int n) {
  const int np = (n + 31) / 32 * 32;
  int g = (n + 127) / 128;
  if (g > 8) g = 8;
  if (g > np / 32) g = np / 32;
  return g < 1 ? 1 : g;
}

// Barrier of the G workgroups sharing one matrix: a counter per matrix
// (zeroed before the launch) that every workgroup raises once per barrier;
// number b waits until it reads G (b + 1). Release on the increment and
// acquire on the polling load, at device scope, carry the workgroups' global
// writes across. The wait is bounded (about a second): should a workgroup
// of the matrix never arrive, the others mark the matrix's diagonal NaN and
// go on, so the kernel always ends.
constexpr int64_t kBarrierSpins = (int64_t)1 << 24;

__device__ void matrix_barrier(int32_t *cnt, int G, int b, double *fail_mark) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const int target = G * (b + 1);
    int64_t spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kBarrierSpins) {
        *fail_mark = __builtin_nan("");
        break;
      }
    }
  }
  __syncthreads();
}

// The reduction of one matrix, by G workgroups (MULTI) or one. With MULTI the
// grid is launched cooperatively (so all its workgroups are resident
// together): the G workgroups of a matrix each form the column, its
// reflector and w-vector redundantly (identical values from identical
// inputs, in a private copy of the panel), split the rows of the
// matrix-vector product between them, and add their partial sums after a
// barrier of the matrix's workgroups, from a buffer that alternates between
// columns; the trailing update's tiles are split between them too, followed
// by a second barrier.
template <bool MULTI, int MAXN>
__device__ void tri_reduce_body(int nmat, int nsec, const int32_t *sec_n, const int32_t *npad,
                                const int64_t *off, double *A, double *work, double *panel,
                                double *xch, bool grouped) {
  // row segments of 64 per lane in A22 v, per pass over the output rows
  constexpr int kAcc = MAXN / 64 < 16 ? MAXN / 64 : 16;
  __shared__ double v[MAXN];
  __shared__ double w[MAXN];
  __shared__ double red[kRedWaves];
  __shared__ double q1[kNb], q2[kNb], vj_s[kNb], wj_s[kNb];
  __shared__ double red_w[kRedWaves / 2][MAXN];
  __shared__ double s_tau, s_scal;
  int mi = blockIdx.x, g = 0, G = 1;
  if (MULTI) {
    int b = blockIdx.x;
    for (mi = 0; mi < nmat; ++mi) {
      G = tri_groups(sec_n[mi % nsec]);
      if (b < G) break;
      b -= G;
    }
    g = b;
  }
  if (!MULTI && mi >= nmat) return;
  // (with MULTI the grid holds exactly the sum of G over the matrices; a
  // surplus workgroup would only take part in the barriers)
  const bool idle = mi >= nmat;
  if (idle) mi = nmat - 1;
  const int n = idle ? 0 : sec_n[mi % nsec];
  const int np = npad[mi];
  const int ncols = n - 2;
  double *Am = A + off[mi];
  double *d = work + off[mi], *e = d + np, *tau = e + np;
  // pending reflectors V[s][row] and w-vectors W[s][row] of the current
  // panel, stored by column so that threads over rows read them coalesced
  double *Vg = panel + off[mi] + (int64_t)g * 2 * kNb * n, *Wg = Vg + (int64_t)n * kNb;
  double *xm = xch + off[mi];   // [2][G][n] partial sums of A22 v
  // barrier counter of the matrix, after d, e, tau and the eigenvalues
  int32_t *cnt = reinterpret_cast<int32_t *>(work + off[mi] + 4 * (int64_t)np);
  int nbar = 0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool lead = (g == 0);
  for (int j0 = 0; j0 < ncols; j0 += kNb) {
    const int jend = min(j0 + kNb, n - 2);   // <= j0: this matrix is done
    const int jlast = min(j0 + kNb, ncols);
    for (int j = j0; j < jlast; ++j) {
      const bool act = j < n - 2;   // uniform over the workgroup
      const int t = j - j0;
      const int m = n - j - 1;
      double tj = 0.0;
      if (act) {
        if (tid < t) {
          vj_s[tid] = Vg[(int64_t)tid * n + j];
          wj_s[tid] = Wg[(int64_t)tid * n + j];
        }
        __syncthreads();
        // column j of the partly reduced matrix: A minus the pending
        // V W^T + W V^T of this panel (row j of A by symmetry)
        double part = 0.0;
        for (int i = tid; i < m; i += kRedThreads) {
          const int64_t r = j + 1 + i;
          double x = Am[(int64_t)j * np + r];
          for (int s2 = 0; s2 < t; ++s2)
            x -= Vg[(int64_t)s2 * n + r] * wj_s[s2] + Wg[(int64_t)s2 * n + r] * vj_s[s2];
          v[i] = x;
          if (i > 0) part += x * x;
        }
        const double sigma = block_sum(part, red);
        if (tid == 0) {
          double dj = Am[(int64_t)j * np + j];
          for (int s2 = 0; s2 < t; ++s2) dj -= 2.0 * vj_s[s2] * wj_s[s2];
          const double alpha = v[0];
          double ej;
          if (sigma == 0.0) {
            s_tau = 0.0;
            s_scal = 0.0;
            ej = alpha;
          } else {
            const double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
            s_tau = (beta - alpha) / beta;
            s_scal = 1.0 / (alpha - beta);
            ej = beta;
          }
          if (lead) {
            d[j] = dj;
            e[j] = ej;
            tau[j] = s_tau;
          }
        }
        __syncthreads();
        tj = s_tau;
      }
      double *vcol = Vg + (int64_t)t * n, *wcol = Wg + (int64_t)t * n;
      const bool refl = act && tj != 0.0;   // uniform over the matrix's workgroups
      if (act && !refl) {   // no reflection: its panel column is zero
        for (int i = tid; i < m; i += kRedThreads) {
          vcol[j + 1 + i] = 0.0;
          wcol[j + 1 + i] = 0.0;
        }
      }
      if (refl) {
        const double sc = s_scal;
        for (int i = tid; i < m; i += kRedThreads) {
          const double vi = (i == 0) ? 1.0 : v[i] * sc;
          v[i] = vi;
          // reflector, for the back-transformation, into row j of A (with
          // MULTI only after the barrier below: the other workgroups of the
          // matrix read row j to form the column)
          if (!MULTI) Am[(int64_t)j * np + j + 1 + i] = vi;
          vcol[j + 1 + i] = vi;
        }
        __syncthreads();
        // q1 = W^T v, q2 = V^T v over the earlier panel columns
        for (int sw = wave; sw < t; sw += kRedWaves) {
          const double *vs = Vg + (int64_t)sw * n + j + 1, *ws = Wg + (int64_t)sw * n + j + 1;
          double a1 = 0.0, a2 = 0.0;
          for (int i = lane; i < m; i += 64) {
            a1 += ws[i] * v[i];
            a2 += vs[i] * v[i];
          }
          a1 = wave_sum(a1);
          a2 = wave_sum(a2);
          if (lane == 0) {
            q1[sw] = a1;
            q2[sw] = a2;
          }
        }
        // A22 v, using the symmetry of A22: sum over k of v[k] times row k,
        // so that lanes run along rows (coalesced) with no cross-lane sums.
        // The k range is split into G x kRedWaves parts (G = tri_groups(n)
        // in a launch whose largest sector has at least kMultiMinRows rows,
        // else 1): group h's kRedWaves
        // parts (one per wave) are added in a fixed order through LDS, then
        // the group sums in order of h. With MULTI group h is workgroup h of
        // the matrix; one workgroup alone runs the groups one after another
        // (grouped; else it takes one group), so both give the same bits.
        const int Gl = MULTI ? 1 : (grouped ? tri_groups(n) : 1);
        const int Gt = MULTI ? G : Gl;
        const double *A22 = Am + (int64_t)(j + 1) * np + (j + 1);
        for (int hh = 0; hh < Gl; ++hh) {
          const int h = MULTI ? g : hh;
          const int part_id = h * kRedWaves + wave, nparts = Gt * kRedWaves;
          const int k_lo = (int)(((int64_t)part_id * m) / nparts);
          const int k_hi = (int)(((int64_t)(part_id + 1) * m) / nparts);
          if constexpr (MAXN <= 1024) {
            double acc[kAcc];
            switch ((m + 63) >> 6) {
#define GXY_MV(Q) \
  case Q: mv_partial<Q>(A22, np, m, k_lo, k_hi, v, lane, acc); break;
              GXY_MV(1) GXY_MV(2) GXY_MV(3) GXY_MV(4) GXY_MV(5) GXY_MV(6) GXY_MV(7) GXY_MV(8)
              GXY_MV(9) GXY_MV(10) GXY_MV(11) GXY_MV(12) GXY_MV(13) GXY_MV(14) GXY_MV(15)
              GXY_MV(16)
#undef GXY_MV
              default: break;
            }
            if (wave >= kRedWaves / 2) {
#pragma unroll
              for (int q = 0; q < kAcc; ++q) {
                const int i = lane + 64 * q;
                if (64 * q < m && i < m) red_w[wave - kRedWaves / 2][i] = acc[q];
              }
            }
            __syncthreads();
            if (wave < kRedWaves / 2) {
#pragma unroll
              for (int q = 0; q < kAcc; ++q) {
                const int i = lane + 64 * q;
                if (64 * q < m && i < m) red_w[wave][i] = acc[q] + red_w[wave][i];
              }
            }
            __syncthreads();
          } else {
            // output rows in passes of 1024 (64 kAcc): the same sums per row
            // as one pass, with half the accumulators per lane (a pass only
            // decides which lanes hold which rows)
            for (int r0 = 0; r0 < m; r0 += 64 * kAcc) {
              const int mr = min(m - r0, 64 * kAcc);
              double acc[kAcc];
              mv_dispatch<64 * kAcc>((mr + 63) >> 6, A22 + r0, np, mr, k_lo, k_hi, v, lane,
                                     acc);
              if (wave >= kRedWaves / 2) {
#pragma unroll
                for (int q = 0; q < kAcc; ++q) {
                  const int i = lane + 64 * q;
                  if (64 * q < mr && i < mr) red_w[wave - kRedWaves / 2][r0 + i] = acc[q];
                }
              }
              __syncthreads();
              if (wave < kRedWaves / 2) {
#pragma unroll
                for (int q = 0; q < kAcc; ++q) {
                  const int i = lane + 64 * q;
                  if (64 * q < mr && i < mr)
                    red_w[wave][r0 + i] = acc[q] + red_w[wave][r0 + i];
                }
              }
              __syncthreads();
            }
          }
          double *xo = xm + ((int64_t)(j & 1) * G + g) * n;
          for (int i = tid; i < m; i += kRedThreads) {
            double x = 0.0;
#pragma unroll
            for (int h8 = 0; h8 < kRedWaves / 2; ++h8) x += red_w[h8][i];
            if (MULTI)
              xo[i] = x;
            else
              w[i] = (hh == 0 ? 0.0 : w[i]) + x;
          }
          __syncthreads();
        }
      }
      if (MULTI) matrix_barrier(cnt, G, nbar++, d);
      if (refl) {
        if (MULTI) {
          const double *xi = xm + (int64_t)(j & 1) * G * n;
          for (int i = tid; i < m; i += kRedThreads) {
            double x = 0.0;
            for (int h = 0; h < G; ++h) x += xi[(int64_t)h * n + i];
            w[i] = x;
            if (lead) Am[(int64_t)j * np + j + 1 + i] = v[i];
          }
        }
        __syncthreads();
        // p = tau (A22 v - V q1 - W q2)
        double pvp = 0.0;
        for (int i = tid; i < m; i += kRedThreads) {
          const int64_t r = j + 1 + i;
          double a = w[i];
          for (int s2 = 0; s2 < t; ++s2)
            a -= Vg[(int64_t)s2 * n + r] * q1[s2] + Wg[(int64_t)s2 * n + r] * q2[s2];
          a *= tj;
          w[i] = a;
          pvp += a * v[i];
        }
        const double K = -0.5 * tj * block_sum(pvp, red);
        for (int i = tid; i < m; i += kRedThreads) wcol[j + 1 + i] = w[i] + K * v[i];
      }
      __syncthreads();
    }
    // trailing matrix (rows and columns >= jend) -= U = V W^T + W V^T, as a
    // K = 32 product on the matrix cores: U[r][c] = sum_k L[r][k] R[c][k]
    // with L[r] = (V[.][r], W[.][r]) and R[c] = (W[.][c], V[.][c]) (zero past
    // the panel width). The waves of the matrix's workgroups take 32 x 32
    // tiles on or below the diagonal and write every new value to (r, c)
    // and (c, r), so A stays exactly symmetric.
    if (jend > j0) {
      const int tp = jend - j0;
      const int mt = n - jend;
      const int nt = (mt + 31) / 32;
      const int ntiles = nt * (nt + 1) / 2;
      const int li = lane & 15, lk = lane >> 4;
      for (int tix = g * kRedWaves + wave; tix < ntiles; tix += G * kRedWaves) {
        int I = (int)((sqrt(8.0 * tix + 1.0) - 1.0) * 0.5);
        while (I * (I + 1) / 2 > tix) --I;
        while ((I + 1) * (I + 2) / 2 <= tix) ++I;
        const int J = tix - I * (I + 1) / 2;
        const int r0 = jend + 32 * I, c0 = jend + 32 * J;
        double4_t acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 32; kk += 4) {
          const int k = kk + lk;
          const int s2 = k & 15;
          const double *Lp = (k < 16 ? Vg : Wg) + (int64_t)s2 * n;
          const double *Rp = (k < 16 ? Wg : Vg) + (int64_t)s2 * n;
          // (columns s2 >= tp of the panel hold stale values: read, then zero)
          double fa[2], fb[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const int r = r0 + 16 * a + li, c = c0 + 16 * a + li;
            const double x = Lp[min(r, n - 1)], y = Rp[min(c, n - 1)];
            fa[a] = (s2 < tp && r < n) ? x : 0.0;
            fb[a] = (s2 < tp && c < n) ? y : 0.0;
          }
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        // accumulator register q of lane l: row l/16 + 4q, column l%16
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int r = r0 + 16 * a + lk + 4 * q, c = c0 + 16 * b + li;
              if (r < n && c < n && (I != J || r >= c)) {
                const double nv = Am[(int64_t)r * np + c] - acc[a][b][q];
                Am[(int64_t)r * np + c] = nv;
                if (r != c) Am[(int64_t)c * np + r] = nv;
              }
            }
      }
    }
    if (MULTI)
      matrix_barrier(cnt, G, nbar++, d);
    else
      __syncthreads();
  }
  if (!idle && tid == 0 && lead) {
    if (n >= 2) {
      d[n - 2] = Am[(int64_t)(n - 2) * np + (n - 2)];
      e[n - 2] = Am[(int64_t)(n - 2) * np + (n - 1)];
      tau[n - 2] = 0.0;
    }
    d[n - 1] = Am[(int64_t)(n - 1) * np + (n - 1)];
    e[n - 1] = 0.0;
    tau[n - 1] = 0.0;
  }
}

template <int MAXN>
__global__ __launch_bounds__(kRedThreads) void tri_reduce_kernel(
    int nmat, int nsec, const int32_t *sec_n, const int32_t *npad, const int64_t *off,
    double *A, double *work, double *panel, int grouped) {
  tri_reduce_body<false, MAXN>(nmat, nsec, sec_n, npad, off, A, work, panel, nullptr,
                               grouped != 0);
}

template <int MAXN>
__global__ __launch_bounds__(kRedThreads) void tri_reduce_multi_kernel(
    int nmat, int nsec, const int32_t *sec_n, const int32_t *npad, const int64_t *off,
    double *A, double *work, double *panel, double *xch) {
  tri_reduce_body<true, MAXN>(nmat, nsec, sec_n, npad, off, A, work, panel, xch, true);
}

// zero the barrier counter of every matrix
__global__ void tri_counters_kernel(int nmat, const int32_t *npad, const int64_t *off,
                                    double *work) {
  const int mi = blockIdx.x * blockDim.x + threadIdx.x;
  if (mi < nmat)
    *reinterpret_cast<int32_t *>(work + off[mi] + 4 * (int64_t)npad[mi]) = 0;
}

// Eigenvalues of T by bisection on Sturm counts (index k = k-th largest).
// The count of eigenvalues below x is the number of negative pivots of the
// LDL^T factorisation of T - x I; pivots smaller than pivmin are replaced by
// -pivmin. Bisection stops when the midpoint no longer lies strictly inside
// the interval, at width max(2 eps |lambda|, eps ||T||) (the absolute floor
// is the usual one of bisection codes: the Householder reduction already
// moves every eigenvalue by about eps ||A||, so halving further only
// resolves rounding noise, at up to 128 halvings for eigenvalues near zero
// instead of about 53), or after 128 halvings. The results are made
// non-increasing in k by tri_values_kernel.
//
// Each eigenvalue has a group of kBisLanes = 2^kBisLevels lanes. The
// midpoints that the next kBisLevels halvings can visit form a binary tree of
// kBisLanes - 1 points, each computed as 0.5 (a + b) from its two enclosing
// points exactly as sequential halving computes it; lane g > 0 takes the
// Sturm count at point g, and every lane of the group then replays the
// halvings (tests included) on the shared counts. The result is the one of
// plain one-point bisection, bit for bit, in a kBisLevels-th of the rounds:
// the Sturm recurrence is a chain of dependent divisions, so the lanes run
// side by side at the latency of one.
constexpr int kBisThreads = 256;
constexpr int kBisLevels = 4;   // bench: 43.2 steps/s against 42.8 with 3
constexpr int kBisLanes = 1 << kBisLevels;
constexpr int kBisPerBlock = kBisThreads / kBisLanes;
constexpr int kBisMaxHalvings = 128;

__device__ int sturm_below(const double *d, const double *e2, int n, double x, double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

template <int MAXN>
__global__ __launch_bounds__(kBisThreads) void tri_bisect_kernel(int nmat, int nsec,
                                                                 const int32_t *sec_n,
                                                                 const int32_t *npad,
                                                                 const int64_t *off,
                                                                 double *work) {
  __shared__ double ds[MAXN], e2s[MAXN];
  __shared__ double red_s[3][kBisThreads / 64];
  const int mi = blockIdx.y;
  if (mi >= nmat) return;
  const int n = sec_n[mi % nsec];
  if (blockIdx.x * kBisPerBlock >= n) return;   // uniform over the block
  const int np = npad[mi];
  double *dg = work + off[mi], *eg = dg + np, *lam = dg + 3 * np;
  // Gershgorin interval and the largest squared off-diagonal (min and max
  // are exact, so the reduction order does not matter)
  double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0;
  for (int i = threadIdx.x; i < n; i += kBisThreads) {
    const double di = dg[i];
    const double el = i > 0 ? eg[i - 1] : 0.0, er = i < n - 1 ? eg[i] : 0.0;
    const double r = fabs(el) + fabs(er);
    ds[i] = di;
    e2s[i] = er * er;
    gl = fmin(gl, di - r);
    gu = fmax(gu, di + r);
    emax2 = fmax(emax2, er * er);
  }
  for (int o = 32; o > 0; o >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, o, 64));
    gu = fmax(gu, __shfl_xor(gu, o, 64));
    emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    red_s[0][threadIdx.x >> 6] = gl;
    red_s[1][threadIdx.x >> 6] = gu;
    red_s[2][threadIdx.x >> 6] = emax2;
  }
  __syncthreads();
  gl = red_s[0][0], gu = red_s[1][0], emax2 = red_s[2][0];
  for (int w = 1; w < kBisThreads / 64; ++w) {
    gl = fmin(gl, red_s[0][w]);
    gu = fmax(gu, red_s[1][w]);
    emax2 = fmax(emax2, red_s[2][w]);
  }
  const double wdt = fmax(gu - gl, DBL_MIN);
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  // absolute floor of the stopping width: eps ||T||, the accuracy to which
  // the reduction itself fixes the eigenvalues
  const double atol = DBL_EPSILON * fmax(fabs(gl), fabs(gu));
  const int g = threadIdx.x % kBisLanes;
  const int k = blockIdx.x * kBisPerBlock + threadIdx.x / kBisLanes;
  if (k >= n) return;   // whole groups leave together
  const int j = n - 1 - k;   // ascending index of the k-th largest eigenvalue
  const int base = (threadIdx.x & 63) & ~(kBisLanes - 1);
  double lo = gl - 2.0 * DBL_EPSILON * wdt - DBL_MIN;
  double hi = gu + 2.0 * DBL_EPSILON * wdt + DBL_MIN;
  int halvings = 0;
  bool done = false;
  while (!done) {
    // this lane's tree point: descend from (lo, hi), halving towards index g
    double x = lo;
    {
      double lv = lo, rv = hi;
      int a = 0;
#pragma unroll
      for (int h = kBisLanes / 2; h >= 1; h >>= 1) {
        const double mv = 0.5 * (lv + rv);
        if (g == a + h) x = mv;
        if (g < a + h) {
          rv = mv;
        } else {
          lv = mv;
          a += h;
        }
      }
    }
    const int c = g > 0 ? sturm_below(ds, e2s, n, x, pivmin) : 0;
    // replay the halvings on the group's points and counts
    int a = 0, z = kBisLanes;
#pragma unroll
    for (int lev = 0; lev < kBisLevels; ++lev) {
      if (halvings == kBisMaxHalvings) {
        done = true;
        break;
      }
      const int m = (a + z) >> 1;
      const double mid = __shfl(x, base + m, 64);
      const int cm = __shfl(c, base + m, 64);
      if (mid <= lo || mid >= hi ||
          hi - lo <= fmax(2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)), atol)) {
        done = true;
        break;
      }
      if (cm > j) {
        z = m;
        hi = mid;
      } else {
        a = m;
        lo = mid;
      }
      ++halvings;
    }
  }
  if (g == 0) lam[k] = 0.5 * (lo + hi);
}

constexpr int kValThreads = 256;

// Make the eigenvalues non-increasing and put them on diag(A) (padding -1),
// where the selection reads them. The reflectors lie right of the diagonal.
template <int MAXN>
__global__ __launch_bounds__(kValThreads) void tri_values_kernel(
    int nmat, int nsec, const int32_t *sec_n, const int32_t *npad, const int64_t *off,
    double *work, double *A) {
  constexpr int kValPer = MAXN / kValThreads;
  const int mi = blockIdx.x;
  if (mi >= nmat) return;
  const int n = sec_n[mi % nsec];
  const int np = npad[mi];
  double *lam = work + off[mi] + 3 * np;
  // prefix minimum (exact, so any grouping gives the same values): each
  // thread scans a run of kValPer, the runs' minima are scanned across the
  // block, then applied. NaN is fmin's identity, so a NaN eigenvalue (a
  // failed reduction) stays where a one-by-one scan would leave it.
  __shared__ double wave_min[kValThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double none = __builtin_nan("");
  double x[kValPer];
  double run = none;
#pragma unroll
  for (int u = 0; u < kValPer; ++u) {
    const int c = tid * kValPer + u;
    run = fmin(run, c < n ? lam[c] : none);
    x[u] = run;
  }
  double incl = run;   // inclusive scan of the run minima over the wave
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(incl, o, 64);
    if (lane >= o) incl = fmin(incl, y);
  }
  if (lane == 63) wave_min[wave] = incl;
  __syncthreads();
  double before = __shfl_up(incl, 1, 64);
  if (lane == 0) before = none;
  for (int w = 0; w < wave; ++w) before = fmin(before, wave_min[w]);
#pragma unroll
  for (int u = 0; u < kValPer; ++u) {
    const int c = tid * kValPer + u;
    if (c < n) lam[c] = fmin(x[u], before);
  }
  __syncthreads();
  double *Am = A + off[mi];
  for (int c = threadIdx.x; c < np; c += blockDim.x)
    Am[(int64_t)c * np + c] = c < n ? lam[c] : -1.0;
}

// Leading kq eigenvectors of T by inverse iteration, one thread per vector:
// three solves of (T - mu I) y = x with the LU factorisation with partial
// pivoting of the tridiagonal matrix, x <- y / max|y| after each, mu the
// eigenvalue, moved apart by pertol = 10 eps ||T|| where consecutive ones are
// closer (so equal eigenvalues give independent solves). Then classical
// Gram-Schmidt, twice, in decreasing eigenvalue order, and unit 2-norm.
// Y[c * np + i]: vector c; U: factor scratch laid out [3][n][kq].
constexpr int kInvThreads = 256;
constexpr int kCgsThreads = 1024;
constexpr int kInvChunk = 8;   // rows per chunk of the factor / solve recurrences
constexpr int kMaxKq = kTriMaxVecs;

__device__ __forceinline__ double start_value(int i, int c) {
  uint64_t z = ((uint64_t)(i + 1) << 32) ^ (uint64_t)(c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

template <int MAXN>
__global__ __launch_bounds__(kInvThreads) void tri_invit_kernel(int nmat, int nsec,
                                                                const int32_t *sec_n,
                                                                const int32_t *npad,
                                                                const int64_t *off,
                                                                const double *work, double *U,
                                                                double *Y, int kmax,
                                                                const double *side) {
  __shared__ double ds[MAXN], es[MAXN];
  __shared__ double mu[kMaxKq];
  __shared__ double tnorm_s;
  const int mi = blockIdx.x;
  if (mi >= nmat) return;
  if (side && (int)*side != mi / nsec) return;   // vectors of the chosen side only
  const int n = sec_n[mi % nsec];
  const int np = npad[mi];
  const int kq = min(min(n, kmax), kMaxKq);
  const double *dg = work + off[mi], *eg = dg + np, *lam = dg + 3 * np;
  double *Um = U + off[mi];
  double *Ym = Y + off[mi];
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += kInvThreads) {
    ds[i] = dg[i];
    es[i] = i < n - 1 ? eg[i] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < n; ++i)
      t = fmax(t, fabs(ds[i]) + fabs(es[i]) + (i > 0 ? fabs(es[i - 1]) : 0.0));
    tnorm_s = fmax(t, DBL_MIN);
    const double pertol = 10.0 * DBL_EPSILON * tnorm_s;
    double prev = 0.0;
    for (int c = 0; c < kq; ++c) {
      double m = lam[c];
      if (c > 0 && prev - m < pertol) m = prev - pertol;
      mu[c] = m;
      prev = m;
    }
  }
  __syncthreads();
  const double tiny = DBL_EPSILON * tnorm_s;
  const bool zero_matrix = tnorm_s <= DBL_MIN;   // any orthonormal basis will do
  // the factor scratch holds 3 n kb doubles (kb vectors at a time) inside
  // this matrix's npad x npad block of U
  const int kb = max(1, min(kq, (int)(((int64_t)np * np) / (3 * (int64_t)n))));
  for (int c0 = 0; c0 < kq; c0 += kb) {
    const int t = tid;
    const int c = c0 + t;
    if (t < kb && c < kq) {
      double *x = Ym + (int64_t)c * np;
      if (n == 1 || zero_matrix) {
        for (int i = 0; i < n; ++i) x[i] = (i == c) ? 1.0 : 0.0;
      } else {
        const double m = mu[c];
        double *u0 = Um, *u1 = Um + (int64_t)n * kb, *u2 = Um + 2 * (int64_t)n * kb;
        for (int i = 0; i < n; ++i) x[i] = start_value(i, c);
        for (int it = 0; it < 3; ++it) {
          // factor T - m I with row interchanges while eliminating the
          // right-hand side x; row i of U is (u0, u1, u2) at columns i..i+2.
          // Rows go in chunks of kInvChunk: the chunk's loads are issued
          // together, its stores after it, so the recurrence waits on
          // memory once per chunk instead of once per row.
          double a = ds[0] - m, bsup = es[0], y = x[0];
          for (int i0 = 0; i0 < n - 1; i0 += kInvChunk) {
            const int cnt = min(kInvChunk, n - 1 - i0);
            double xn[kInvChunk], o0[kInvChunk], o1[kInvChunk], o2[kInvChunk], ox[kInvChunk];
#pragma unroll
            for (int q = 0; q < kInvChunk; ++q) xn[q] = x[min(i0 + q + 1, n - 1)];
#pragma unroll
            for (int q = 0; q < kInvChunk; ++q) {
              if (q < cnt) {
                const int i = i0 + q;
                const double csub = es[i];            // T[i+1][i]
                const double anext = ds[i + 1] - m;   // T[i+1][i+1]
                const double bnext = i + 1 < n - 1 ? es[i + 1] : 0.0;
                const double ynext = xn[q];
                if (fabs(a) >= fabs(csub)) {
                  const double piv = (a != 0.0) ? a : tiny;
                  const double l = csub / piv;
                  o0[q] = piv;
                  o1[q] = bsup;
                  o2[q] = 0.0;
                  ox[q] = y;
                  a = anext - l * bsup;
                  bsup = bnext;
                  y = ynext - l * y;
                } else {
                  const double l = a / csub;
                  o0[q] = csub;
                  o1[q] = anext;
                  o2[q] = bnext;
                  ox[q] = ynext;
                  a = bsup - l * anext;
                  bsup = -l * bnext;
                  y = y - l * ynext;
                }
              }
            }
#pragma unroll
            for (int q = 0; q < kInvChunk; ++q) {
              if (q < cnt) {
                const int64_t at = (int64_t)(i0 + q) * kb + t;
                u0[at] = o0[q];
                u1[at] = o1[q];
                u2[at] = o2[q];
                x[i0 + q] = ox[q];
              }
            }
          }
          {
            const int64_t at = (int64_t)(n - 1) * kb + t;
            u0[at] = (a != 0.0) ? a : tiny;
            x[n - 1] = y;
          }
          // back substitution (rows in chunks as above), then scale by the
          // largest entry
          double xmax = 0.0, x1 = 0.0, x2 = 0.0;
          for (int i1 = n - 1; i1 >= 0; i1 -= kInvChunk) {
            const int cnt = min(kInvChunk, i1 + 1);
            double b0[kInvChunk], b1[kInvChunk], b2[kInvChunk], bx[kInvChunk];
#pragma unroll
            for (int q = 0; q < kInvChunk; ++q) {
              const int i = max(i1 - q, 0);
              const int64_t at = (int64_t)i * kb + t;
              b0[q] = u0[at];
              b1[q] = u1[at];
              b2[q] = u2[at];
              bx[q] = x[i];
            }
#pragma unroll
            for (int q = 0; q < kInvChunk; ++q) {
              if (q < cnt) {
                const double v = (bx[q] - b1[q] * x1 - b2[q] * x2) / b0[q];
                bx[q] = v;
                x2 = x1;
                x1 = v;
                xmax = fmax(xmax, fabs(v));
              }
            }
#pragma unroll
            for (int q = 0; q < kInvChunk; ++q)
              if (q < cnt) x[i1 - q] = bx[q];
          }
          // (in chunks too: one element at a time, each load would wait)
          const double inv = xmax > 0.0 ? 1.0 / xmax : 1.0;
          for (int i0 = 0; i0 < n; i0 += kInvChunk) {
            double xs[kInvChunk];
#pragma unroll
            for (int q = 0; q < kInvChunk; ++q) xs[q] = x[min(i0 + q, n - 1)];
#pragma unroll
            for (int q = 0; q < kInvChunk; ++q)
              if (i0 + q < n) x[i0 + q] = xs[q] * inv;
          }
        }
      }
    }
    __syncthreads();
  }
}

// Classical Gram-Schmidt, twice, over the inverse-iteration vectors of a
// matrix, in order c = 0, 1, ...; the vector being orthogonalised stays in
// LDS over its two passes; 16 waves take the dot products.
template <int MAXN>
__global__ __launch_bounds__(kCgsThreads) void tri_cgs_kernel(int nmat, int nsec,
                                                             const int32_t *sec_n,
                                                             const int32_t *npad,
                                                             const int64_t *off, double *Y,
                                                             int kmax, const double *side) {
  __shared__ double xs[MAXN];
  __shared__ double dot[kMaxKq];
  __shared__ double red[kCgsThreads / 64];
  const int mi = blockIdx.x;
  if (mi >= nmat) return;
  if (side && (int)*side != mi / nsec) return;
  const int n = sec_n[mi % nsec];
  const int np = npad[mi];
  const int kq = min(min(n, kmax), kMaxKq);
  double *Ym = Y + off[mi];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c = 0; c < kq; ++c) {
    double *xc = Ym + (int64_t)c * np;
    for (int i = tid; i < n; i += kCgsThreads) xs[i] = xc[i];
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = wave; j < c; j += kCgsThreads / 64) {
        const double *xj = Ym + (int64_t)j * np;
        double acc = 0.0;
        // (unrolled: the loads of several rows are issued before the
        // accumulation, which keeps its order)
#pragma unroll 8
        for (int i = lane; i < n; i += 64) acc += xj[i] * xs[i];
        acc = wave_sum(acc);
        if (lane == 0) dot[j] = acc;
      }
      __syncthreads();
      for (int i = tid; i < n; i += kCgsThreads) {
        double v = xs[i];
#pragma unroll 8
        for (int j = 0; j < c; ++j) v -= dot[j] * Ym[(int64_t)j * np + i];
        xs[i] = v;
      }
      __syncthreads();
    }
    double part = 0.0;
    for (int i = tid; i < n; i += kCgsThreads) part += xs[i] * xs[i];
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    double nrm2 = 0.0;
    for (int w = 0; w < kCgsThreads / 64; ++w) nrm2 += red[w];
    const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
    for (int i = tid; i < n; i += kCgsThreads) xc[i] = xs[i] * inv;
    __syncthreads();
  }
}

// Eigenvalues to diag(A); the leading kq eigenvectors of A = H Y, with
// H = H_0 H_1 ... H_{n-3} (the last reflector applied first), written to V.
// Columns are independent: workgroup (x, mi) takes columns x*16 .. x*16+15,
// one per wave, so the waves never wait for each other.
// Workgroup shape by size: up to 1024 rows 1024 threads and blocks of 16
// reflectors; up to 2048 rows 512 threads (a wave then holds 2 x 32 values
// per lane) and blocks of 4 (the LDS stage stays at 64 KB). The blocking
// only stages the reflectors: each column goes through them one by one in
// the same order either way.
template <int MAXN> struct BackShape {
  static constexpr int threads = MAXN <= 1024 ? 1024 : 512;
  static constexpr int blk = MAXN <= 1024 ? 16 : 4;
  static constexpr int cols = threads / 64;
};

// One wave's column y (held in registers: lane l keeps rows l + 64 q, q < Q)
// through the reflectors j = n-3 .. 0, in blocks of BackShape::blk staged in
// LDS by the whole workgroup (vb[t][r] = v_j[r] for r > j, else 0).
template <int Q, int MAXN>
__device__ __forceinline__ void back_column(const double *Am, const double *tau, int n, int np,
                                            double *yc, bool active, double (*vb)[MAXN],
                                            int lane, int tid) {
  constexpr int kBackBlk = BackShape<MAXN>::blk, kBackThreads = BackShape<MAXN>::threads;
  double y[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = lane + 64 * q;
    y[q] = (active && r < n) ? yc[r] : 0.0;
  }
  for (int jb = n - 3; jb >= 0; jb -= kBackBlk) {
    const int nb = min(kBackBlk, jb + 1);   // reflectors jb, jb-1, .., jb-nb+1
    __syncthreads();
    for (int e = tid; e < nb * n; e += kBackThreads) {
      const int t = e / n, r = e % n;
      const int j = jb - t;
      vb[t][r] = r > j ? Am[(int64_t)j * np + r] : 0.0;
    }
    __syncthreads();
    if (active) {
      for (int t = 0; t < nb; ++t) {
        const double tj = tau[jb - t];
        if (tj == 0.0) continue;
        double vv[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int r = lane + 64 * q;
          vv[q] = r < n ? vb[t][min(r, n - 1)] : 0.0;
        }
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) acc += vv[q] * y[q];
        const double sdot = tj * wave_sum(acc);
#pragma unroll
        for (int q = 0; q < Q; ++q) y[q] -= sdot * vv[q];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = lane + 64 * q;
    if (active && r < n) yc[r] = y[q];
  }
}

template <int Q, int MAXN>
__device__ void back_dispatch(int nq, const double *Am, const double *tau, int n, int np,
                              double *yc, bool active, double (*vb)[MAXN], int lane, int tid) {
  if constexpr (Q <= MAXN / 64) {
    if (nq == Q) {
      back_column<Q, MAXN>(Am, tau, n, np, yc, active, vb, lane, tid);
      return;
    }
    back_dispatch<Q + 1, MAXN>(nq, Am, tau, n, np, yc, active, vb, lane, tid);
  }
}

template <int MAXN>
__global__ __launch_bounds__(BackShape<MAXN>::threads) void tri_back_kernel(
    int nmat, int nsec, const int32_t *sec_n, const int32_t *npad, const int64_t *off,
    const double *A, const double *work, double *V, double *Y, int kmax, const double *side) {
  constexpr int kBackThreads = BackShape<MAXN>::threads, kBackCols = BackShape<MAXN>::cols;
  __shared__ double vb[BackShape<MAXN>::blk][MAXN];
  const int mi = blockIdx.y;
  if (mi >= nmat) return;
  if (side && (int)*side != mi / nsec) return;
  const int n = sec_n[mi % nsec];
  const int np = npad[mi];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double *dg = work + off[mi], *tau = dg + 2 * np;
  const double *Am = A + off[mi];
  double *Vm = V + off[mi];
  double *Ym = Y + off[mi];   // Y[c * np + r], c < kq
  const int kq = min(min(n, kmax), kMaxKq);
  const int c = blockIdx.x * kBackCols + wave;
  const bool active = c < kq;
  double *yc = Ym + (int64_t)(active ? c : 0) * np;
  back_dispatch<1, MAXN>((n + 63) >> 6, Am, tau, n, np, yc, active, vb, lane, tid);
  __syncthreads();
  if (active)
    for (int r = lane; r < n; r += 64) Vm[(int64_t)r * np + c] = yc[r];
  if (blockIdx.x == 0) {
    // columns kq .. np-1 of V are zero
    for (int64_t el = tid; el < (int64_t)n * (np - kq); el += kBackThreads) {
      const int r = (int)(el / (np - kq)), cc = kq + (int)(el % (np - kq));
      Vm[(int64_t)r * np + cc] = 0.0;
    }
  }
}

// co-resident workgroups of the multi-workgroup kernel (per process, one
// device type; 0 without cooperative launch)
template <int MAXN>
int co_resident() {
  static const int n = []() {
    int dev = 0, per_cu = 0, cus = 0, coop = 0;
    GXY_HIP(hipGetDevice(&dev));
    GXY_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    GXY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    GXY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(tri_reduce_multi_kernel<MAXN>), kRedThreads, 0));
    return coop ? per_cu * cus : 0;
  }();
  return n;
}

template <int MAXN>
void tri_values_impl(int nmat, int nsec, const int *h_sec_n, const int32_t *d_sec_n,
                     const int32_t *d_npad, const int64_t *d_off, double *A, double *Y,
                     double *X, double *work, bool allow_multi, hipStream_t s) {
  // Y serves as the panel scratch of the reduction (G private panels of
  // 2 n kNb values per matrix <= npad^2), X as the exchange of partial
  // matrix-vector products (2 G n <= npad^2)
  int blocks = 0, ncols = 0;
  for (int k = 0; k < nmat; ++k) {
    const int n = h_sec_n[k % nsec];
    blocks += tri_groups(n);
    ncols = std::max(ncols, n - 2);
  }
  const char *env = getenv("GXY_TRI_MULTI");
  // (a launch whose largest sector qualifies groups the sums the shared way
  // even on one workgroup per matrix, so the bits do not depend on whether
  // the cooperative launch was possible)
  const char *env_min = getenv("GXY_TRI_MULTI_MIN");   // rows; default kMultiMinRows
  const int min_rows = env_min ? atoi(env_min) : kMultiMinRows;
  const bool grouped = ncols + 2 >= min_rows;
  const bool multi = allow_multi && !(env && env[0] == '0') && grouped && blocks > nmat &&
                     blocks <= co_resident<MAXN>();
  if (multi) {
    hipLaunchKernelGGL(tri_counters_kernel, dim3((nmat + 255) / 256), dim3(256), 0, s, nmat,
                       d_npad, d_off, work);
    GXY_CHECK_LAUNCH();
    // The workgroups of a matrix wait for each other, so the whole grid must
    // be resident at once: the cooperative launch has the runtime promise
    // that. The grid is sized to fit an idle device (co_resident), and the
    // other kernels' workgroups end by themselves, so a regular launch of the
    // same grid (GXY_TRI_COOP=0) gets there too, with the same values and
    // speed, for tools that fail on cooperative launches. (Neither form is
    // meant for two such reductions at once: batch workers never share.)
    const char *coop = getenv("GXY_TRI_COOP");
    if (coop && coop[0] == '0') {
      hipLaunchKernelGGL(tri_reduce_multi_kernel<MAXN>, dim3(blocks), dim3(kRedThreads), 0, s,
                         nmat, nsec, d_sec_n, d_npad, d_off, A, work, Y, X);
      GXY_CHECK_LAUNCH();
    } else {
      void *args[] = {&nmat, &nsec, &d_sec_n, &d_npad, &d_off, &A, &work, &Y, &X};
      GXY_HIP(hipLaunchCooperativeKernel(
          reinterpret_cast<const void *>(tri_reduce_multi_kernel<MAXN>), dim3(blocks),
          dim3(kRedThreads), args, 0, s));
    }
  } else {
    hipLaunchKernelGGL(tri_reduce_kernel<MAXN>, dim3(nmat), dim3(kRedThreads), 0, s, nmat, nsec,
                       d_sec_n, d_npad, d_off, A, work, Y, grouped ? 1 : 0);
    GXY_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(tri_bisect_kernel<MAXN>, dim3(MAXN / kBisPerBlock, nmat),
                     dim3(kBisThreads), 0, s, nmat, nsec, d_sec_n, d_npad, d_off, work);
  GXY_CHECK_LAUNCH();
  hipLaunchKernelGGL(tri_values_kernel<MAXN>, dim3(nmat), dim3(kValThreads), 0, s, nmat, nsec,
                     d_sec_n, d_npad, d_off, work, A);
  GXY_CHECK_LAUNCH();
}

template <int MAXN>
void tri_vectors_impl(int nmat, int nsec, const int32_t *d_sec_n, const int32_t *d_npad,
                      const int64_t *d_off, const double *A, double *V, double *Y,
                      const double *work, int kmax, const double *d_side, hipStream_t s) {
  // V serves as the factor scratch of the inverse iteration until tri_back
  hipLaunchKernelGGL(tri_invit_kernel<MAXN>, dim3(nmat), dim3(kInvThreads), 0, s, nmat, nsec,
                     d_sec_n, d_npad, d_off, work, V, Y, kmax, d_side);
  GXY_CHECK_LAUNCH();
  hipLaunchKernelGGL(tri_cgs_kernel<MAXN>, dim3(nmat), dim3(kCgsThreads), 0, s, nmat, nsec,
                     d_sec_n, d_npad, d_off, Y, kmax, d_side);
  GXY_CHECK_LAUNCH();
  constexpr int cols = BackShape<MAXN>::cols;
  const int nx = (std::min(kmax, kMaxKq) + cols - 1) / cols;
  hipLaunchKernelGGL(tri_back_kernel<MAXN>, dim3(std::max(nx, 1), nmat),
                     dim3(BackShape<MAXN>::threads), 0, s, nmat, nsec, d_sec_n, d_npad, d_off, A,
                     work, V, Y, kmax, d_side);
  GXY_CHECK_LAUNCH();
}

}  // namespace

// The kernels are instantiated for matrices of up to 1024 and up to
// kTriMaxN = 2048 rows; a launch takes the smaller instantiation that holds
// its largest sector (the arithmetic is the same in both, so the choice
// changes no value).
void launch_tri_values(int nmat, int nsec, const int *h_sec_n, const int32_t *d_sec_n,
                       const int32_t *d_npad, const int64_t *d_off, double *A, double *Y,
                       double *X, double *work, bool allow_multi, hipStream_t s) {
  int maxn = 0;
  for (int k = 0; k < nsec; ++k) maxn = std::max(maxn, h_sec_n[k]);
  if (maxn > kTriMaxN) fail(GXY_EUNSUPPORTED, "tridiagonal path: sector above 2048 rows");
  if (maxn <= 1024)
    tri_values_impl<1024>(nmat, nsec, h_sec_n, d_sec_n, d_npad, d_off, A, Y, X, work,
                          allow_multi, s);
  else
    tri_values_impl<kTriMaxN>(nmat, nsec, h_sec_n, d_sec_n, d_npad, d_off, A, Y, X, work,
                              allow_multi, s);
}

void launch_tri_vectors(int nmat, int nsec, int maxn, const int32_t *d_sec_n,
                        const int32_t *d_npad, const int64_t *d_off, const double *A, double *V,
                        double *Y, const double *work, int kmax, const double *d_side,
                        hipStream_t s) {
  if (kmax > kMaxKq) fail(GXY_EUNSUPPORTED, "tridiagonal path: more than 128 vectors");
  if (maxn > kTriMaxN) fail(GXY_EUNSUPPORTED, "tridiagonal path: sector above 2048 rows");
  if (maxn <= 1024)
    tri_vectors_impl<1024>(nmat, nsec, d_sec_n, d_npad, d_off, A, V, Y, work, kmax, d_side, s);
  else
    tri_vectors_impl<kTriMaxN>(nmat, nsec, d_sec_n, d_npad, d_off, A, V, Y, work, kmax, d_side,
                               s);
}

}  // namespace gxy
