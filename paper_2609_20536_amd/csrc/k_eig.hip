// Batched FP64 symmetric eigensolver: two-sided block Jacobi.
//
// The HOSVD factors U and V of M (Ch. 2, eq. hosvd) are the eigenvectors of
// the Gram matrices of M's left and right unfoldings; the eigenvalues are the
// squared mode norms |S_{i,:,:,:}|^2 that enter the discarded weights. The
// Gram matrix is block diagonal in the symmetry label of the fused bond, so
// every label sector of both sides is one matrix of the batch.
//
// Each matrix is padded to a multiple of 32 rows (padding: -1 on the diagonal,
// zero coupling, so it never mixes with the real block) and split into
// 16-row blocks. One outer round pairs all blocks (round-robin / circle
// order); every pair's 32x32 subproblem is diagonalised completely by a
// cyclic Jacobi in LDS by one wave, and the resulting rotation is applied to
// the pair's block rows and columns and accumulated into V. nb-1 rounds
// make a sweep; sweeps repeat until no pair has a significant coupling.
#include "internal.h"

namespace gxy {

namespace {

constexpr int kB = 16;          // block size
constexpr int kP = 2 * kB;      // pair subproblem size
// A coupling a_pq is rotated away only if |a_pq| > abs_tol * scale and
// |a_pq| > rel_tol * sqrt(|a_pp a_qq|), scale being the largest diagonal entry
// over every matrix of the batch (the accuracy class of a backward stable
// solver is eps * ||E||). The tolerances are arguments: a loose first stage,
// a tight refinement stage.

// Blocks of pair p in round r for nb blocks (circle method: block 0 fixed).
__device__ inline void pair_blocks(int nb, int r, int p, int &bi, int &bj) {
  if (nb == 2) {
    bi = 0;
    bj = 1;
    return;
  }
  const int m = nb - 1;
  const int rr = r % m;
  auto block_at = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + rr) % m) + 1; };
  bi = block_at(p);
  bj = block_at(nb - 1 - p);
  if (bi > bj) {
    const int t = bi;
    bi = bj;
    bj = t;
  }
}

__device__ inline int pair_row(int a, int bi, int bj) {
  return a < kB ? bi * kB + a : bj * kB + (a - kB);
}

// inner pairing of 32 indices (circle method, index 0 fixed)
__device__ inline void inner_pair(int r, int p, int &a, int &b) {
  const int m = kP - 1;
  auto at = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + r) % m) + 1; };
  a = at(p);
  b = at(kP - 1 - p);
}

__global__ void eig_gather_kernel(const double *E, int nfused, const int32_t *sec_idx,
                                  const int32_t *sec_start, const int32_t *sec_n,
                                  int nsec, int nmat, const int32_t *npad,
                                  const int64_t *off, double *A, double *V,
                                  int side_stride_elems) {
  // blockIdx.y = matrix, grid-stride over its elements
  const int mi = blockIdx.y;
  if (mi >= nmat) return;
  const int side = mi / nsec;
  const int s = mi % nsec;
  const double *Es = E + (int64_t)side * side_stride_elems;
  const int n = sec_n[s];
  const int np = npad[mi];
  const int st = sec_start[s];
  double *Am = A + off[mi];
  double *Vm = V ? V + off[mi] : Am;
  const int64_t tot = (int64_t)np * np;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / np), j = (int)(e % np);
    double v;
    if (i < n && j < n)
      v = Es[(int64_t)sec_idx[st + i] * nfused + sec_idx[st + j]];
    else
      v = (i == j) ? -1.0 : 0.0;
    Am[e] = v;
    if (Vm != Am) Vm[e] = (i == j) ? 1.0 : 0.0;
  }
}

// global scale: max over matrices, written to every entry
__global__ void eig_scale_max_kernel(int nmat, double *scale) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < nmat; i += 256) m = fmax(m, scale[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const double g = red[0];
  __syncthreads();
  for (int i = threadIdx.x; i < nmat; i += 256) scale[i] = g;
}

__global__ void eig_scale_kernel(const int32_t *npad, const int64_t *off,
                                 const double *A, double *scale, int32_t *flags) {
  __shared__ double red[256];
  const int mi = blockIdx.x;
  const int np = npad[mi];
  const double *Am = A + off[mi];
  double m = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) m = fmax(m, fabs(Am[(int64_t)i * np + i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scale[mi] = red[0];
    flags[mi] = 1;
  }
}

// One workgroup (4 waves) per pair: one cyclic sweep over the 32x32
// subproblem, written back in place, and the accumulated rotation Q
// (32x32, row-major). A pair without a significant coupling is left alone
// (pair_rot = 0) so the update kernel can skip it.
constexpr int kSolveThreads = 256;

__global__ __launch_bounds__(kSolveThreads) void eig_solve_kernel(
    int round, int total_pairs, const int32_t *pair_mat, const int32_t *pairbase,
    const int32_t *npad, const int64_t *off, double *A, double *Qbuf, const double *scale,
    int32_t *flags, int32_t *next_flags, double abs_tol, double rel_tol, double gap_tol,
    int inner_sweeps, int32_t *pair_rot) {
  __shared__ double S[kP][kP + 1];
  __shared__ double Qs[kP][kP + 1];
  __shared__ double cs[kP / 2][2];
  __shared__ int ab[kP / 2][2];
  __shared__ int any_rot;
  const int pid = blockIdx.x;
  if (pid >= total_pairs) return;
  const int mi = pair_mat[pid];
  const int p = pid - pairbase[mi];
  const int np = npad[mi];
  const int nb = np / kB;
  double *Qp = Qbuf + (int64_t)pid * kP * kP;
  const int tid = threadIdx.x;
  if (flags[mi] == 0) {
    if (tid == 0) pair_rot[pid] = 0;
    return;
  }
  int bi, bj;
  pair_blocks(nb, round, p, bi, bj);
  double *Am = A + off[mi];
  for (int e = tid; e < kP * kP; e += kSolveThreads) {
    const int a = e / kP, b = e % kP;
    const int ra = pair_row(a, bi, bj), rb = pair_row(b, bi, bj);
    // symmetrise: average the two triangles
    S[a][b] = 0.5 * (Am[(int64_t)ra * np + rb] + Am[(int64_t)rb * np + ra]);
    Qs[a][b] = (a == b) ? 1.0 : 0.0;
  }
  if (tid == 0) any_rot = 0;
  __syncthreads();
  const double absthr = abs_tol * scale[mi];
  const double floor_thr = 1e-20 * scale[mi];
  // a coupling is rotated away if it is above the rounding noise of its own
  // entries (rel_tol) and either large in absolute terms (abs_tol) or large
  // against the gap of its diagonal pair (gap_tol: rotation angle)
  auto significant = [&](double apq, double app, double aqq) {
    const double x = fabs(apq);
    return x > floor_thr && x > rel_tol * sqrt(fabs(app * aqq)) &&
           (x > absthr || x > gap_tol * fabs(app - aqq));
  };
  int sig = 0;
  for (int e = tid; e < kP * kP; e += kSolveThreads) {
    const int a = e / kP, b = e % kP;
    if (a != b && significant(S[a][b], S[a][a], S[b][b])) sig = 1;
  }
  if (sig) any_rot = 1;
  __syncthreads();
  if (!any_rot) {
    if (tid == 0) pair_rot[pid] = 0;
    return;
  }
  if (tid == 0) {
    next_flags[mi] = 1;
    pair_rot[pid] = 1;
  }
  for (int sweep = 0; sweep < inner_sweeps; ++sweep) {
    for (int r = 0; r < kP - 1; ++r) {
      if (tid < kP / 2) {
        int a, b;
        inner_pair(r, tid, a, b);
        if (a > b) {
          const int t = a;
          a = b;
          b = t;
        }
        const double apq = S[a][b];
        const double app = S[a][a], aqq = S[b][b];
        double c = 1.0, s = 0.0;
        if (significant(apq, app, aqq)) {
          const double tau = (aqq - app) / (2.0 * apq);
          double t;
          if (fabs(tau) > 1e150)
            t = 0.5 / tau;
          else
            t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        cs[tid][0] = c;
        cs[tid][1] = s;
        ab[tid][0] = a;
        ab[tid][1] = b;
      }
      __syncthreads();
      // rows: (row_a, row_b) <- (c row_a - s row_b, s row_a + c row_b)
      for (int e = tid; e < (kP / 2) * kP; e += kSolveThreads) {
        const int q = e / kP, k = e % kP;
        const double c = cs[q][0], s = cs[q][1];
        if (s == 0.0) continue;
        const int a = ab[q][0], b = ab[q][1];
        const double xa = S[a][k], xb = S[b][k];
        S[a][k] = c * xa - s * xb;
        S[b][k] = s * xa + c * xb;
      }
      __syncthreads();
      // columns of S and of Q
      for (int e = tid; e < (kP / 2) * kP; e += kSolveThreads) {
        const int q = e / kP, k = e % kP;
        const double c = cs[q][0], s = cs[q][1];
        if (s == 0.0) continue;
        const int a = ab[q][0], b = ab[q][1];
        const double xa = S[k][a], xb = S[k][b];
        S[k][a] = c * xa - s * xb;
        S[k][b] = s * xa + c * xb;
        const double qa = Qs[k][a], qb = Qs[k][b];
        Qs[k][a] = c * qa - s * qb;
        Qs[k][b] = s * qa + c * qb;
      }
      __syncthreads();
      if (tid < kP / 2 && cs[tid][1] != 0.0) {
        const int a = ab[tid][0], b = ab[tid][1];
        S[a][b] = 0.0;
        S[b][a] = 0.0;
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < kP * kP; e += kSolveThreads) {
    const int a = e / kP, b = e % kP;
    Qp[e] = Qs[a][b];
    const int ra = pair_row(a, bi, bj), rb = pair_row(b, bi, bj);
    Am[(int64_t)ra * np + rb] = S[a][b];
  }
}

// Update tiles. Descriptor (mat, kind, x, y): kind 0 -> A[pair x, pair y]
// (x < y) and its transpose; kind 1 -> V[row block x (32 rows), pair y].
__global__ __launch_bounds__(256) void eig_update_kernel(int round, const int32_t *tiles,
                                                         int ntiles,
                                                         const int32_t *pairbase,
                                                         const int32_t *npad,
                                                         const int64_t *off, double *A,
                                                         double *V, const double *Qbuf,
                                                         const int32_t *flags,
                                                         const int32_t *pair_rot) {
  __shared__ double X[kP][kP + 1];
  __shared__ double Qx[kP][kP + 1];
  __shared__ double Qy[kP][kP + 1];
  __shared__ double T1[kP][kP + 1];
  const int t = blockIdx.x;
  if (t >= ntiles) return;
  const int mi = tiles[4 * t], kind = tiles[4 * t + 1];
  const int x = tiles[4 * t + 2], y = tiles[4 * t + 3];
  if (flags[mi] == 0) return;
  const int32_t *rot = pair_rot + pairbase[mi];
  if (!rot[y] && (kind == 1 || !rot[x])) return;  // nothing rotated in these pairs
  const int np = npad[mi];
  const int nb = np / kB;
  const int tid = threadIdx.x;
  int yi, yj;
  pair_blocks(nb, round, y, yi, yj);
  const double *Qyp = Qbuf + (int64_t)(pairbase[mi] + y) * kP * kP;
  for (int e = tid; e < kP * kP; e += 256)
    Qy[e / kP][e % kP] = rot[y] ? Qyp[e] : (e / kP == e % kP ? 1.0 : 0.0);
  if (kind == 0) {
    int xi, xj;
    pair_blocks(nb, round, x, xi, xj);
    const double *Qxp = Qbuf + (int64_t)(pairbase[mi] + x) * kP * kP;
    double *Am = A + off[mi];
    for (int e = tid; e < kP * kP; e += 256) {
      const int a = e / kP, b = e % kP;
      Qx[a][b] = rot[x] ? Qxp[e] : (a == b ? 1.0 : 0.0);
      X[a][b] = Am[(int64_t)pair_row(a, xi, xj) * np + pair_row(b, yi, yj)];
    }
    __syncthreads();
    // T1 = Qx^T X
    for (int e = tid; e < kP * kP; e += 256) {
      const int a = e / kP, b = e % kP;
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < kP; ++k) acc += Qx[k][a] * X[k][b];
      T1[a][b] = acc;
    }
    __syncthreads();
    // out = T1 Qy, written to A[x, y] and transposed to A[y, x]
    for (int e = tid; e < kP * kP; e += 256) {
      const int a = e / kP, b = e % kP;
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < kP; ++k) acc += T1[a][k] * Qy[k][b];
      const int ra = pair_row(a, xi, xj), cb = pair_row(b, yi, yj);
      Am[(int64_t)ra * np + cb] = acc;
      Am[(int64_t)cb * np + ra] = acc;
    }
  } else {
    double *Vm = V + off[mi];
    const int r0 = x * kP;
    for (int e = tid; e < kP * kP; e += 256) {
      const int a = e / kP, b = e % kP;
      X[a][b] = Vm[(int64_t)(r0 + a) * np + pair_row(b, yi, yj)];
    }
    __syncthreads();
    for (int e = tid; e < kP * kP; e += 256) {
      const int a = e / kP, b = e % kP;
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < kP; ++k) acc += X[a][k] * Qy[k][b];
      Vm[(int64_t)(r0 + a) * np + pair_row(b, yi, yj)] = acc;
    }
  }
}

__global__ void eig_identity_kernel(int nmat, const int32_t *npad, const int64_t *off,
                                    double *V) {
  const int mi = blockIdx.y;
  if (mi >= nmat) return;
  const int np = npad[mi];
  double *Vm = V + off[mi];
  const int64_t tot = (int64_t)np * np;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x)
    Vm[e] = (e / np == e % np) ? 1.0 : 0.0;
}

__global__ void eig_axpby_kernel(int64_t n, double a, const double *x, double *y) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    y[i] = a * x[i];
}

}  // namespace

void launch_eig_identity(const EigBatch &b, double *V, hipStream_t s) {
  hipLaunchKernelGGL(eig_identity_kernel, dim3(64, b.nmat), dim3(256), 0, s, b.nmat, b.d_npad,
                     b.d_off, V);
  GXY_CHECK_LAUNCH();
}

void launch_eig_scaled_copy(int64_t n, double a, const double *x, double *y, hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(eig_axpby_kernel, dim3((unsigned)g), dim3(256), 0, s, n, a, x, y);
  GXY_CHECK_LAUNCH();
}

void launch_eig_gather(const double *E, int nfused, const int32_t *d_sec_idx,
                       const int32_t *d_sec_start, const int32_t *d_sec_n, int nsec,
                       const EigBatch &b, hipStream_t s) {
  dim3 grid(64, b.nmat);
  hipLaunchKernelGGL(eig_gather_kernel, grid, dim3(256), 0, s, E, nfused, d_sec_idx,
                     d_sec_start, d_sec_n, nsec, b.nmat, b.d_npad, b.d_off, b.A, b.V,
                     nfused * nfused);
  GXY_CHECK_LAUNCH();
}

void launch_eig_scale(const EigBatch &b, hipStream_t s) {
  hipLaunchKernelGGL(eig_scale_kernel, dim3(b.nmat), dim3(256), 0, s, b.d_npad, b.d_off,
                     b.A, b.d_scale, b.d_flags);
  GXY_CHECK_LAUNCH();
  hipLaunchKernelGGL(eig_scale_max_kernel, dim3(1), dim3(256), 0, s, b.nmat, b.d_scale);
  GXY_CHECK_LAUNCH();
}

void launch_eig_round(const EigBatch &b, int round, double abs_tol, double rel_tol,
                      double gap_tol, int inner_sweeps, hipStream_t s) {
  // flags: d_flags[0..nmat) current sweep, d_flags[nmat..2nmat) next sweep
  hipLaunchKernelGGL(eig_solve_kernel, dim3(b.total_pairs), dim3(kSolveThreads), 0, s,
                     round, b.total_pairs, b.d_pair_mat, b.d_pairbase, b.d_npad, b.d_off, b.A,
                     b.Q, b.d_scale, b.d_flags, b.d_flags + b.nmat, abs_tol, rel_tol,
                     gap_tol, inner_sweeps, b.d_pair_rot);
  GXY_CHECK_LAUNCH();
  if (b.n_update_tiles > 0) {
    hipLaunchKernelGGL(eig_update_kernel, dim3(b.n_update_tiles), dim3(256), 0, s, round,
                       b.d_rtl, b.n_update_tiles, b.d_pairbase, b.d_npad, b.d_off, b.A,
                       b.V, b.Q, b.d_flags, b.d_pair_rot);
    GXY_CHECK_LAUNCH();
  }
}

}  // namespace gxy
