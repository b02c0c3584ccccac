// Internal declarations shared by the HIP sources of libgxyhotrg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gxy_hotrg.h"
#include "../../include/gxy_lgt.h"

namespace gxy {

// --------------------------------------------------------------------------
// errors
// --------------------------------------------------------------------------

struct Error {
  gxy_status status;
  std::string msg;
};

#define GXY_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      throw ::gxy::Error{GXY_EDEVICE, std::string(#call) + ": " +            \
                                          hipGetErrorString(e_)};            \
  } while (0)

#define GXY_CHECK_LAUNCH() GXY_HIP(hipGetLastError())

[[noreturn]] inline void fail(gxy_status s, const std::string &m) {
  throw Error{s, m};
}

// --------------------------------------------------------------------------
// Mixed-radix index maps: a fused index x = ((d0 * e1 + d1) * e2 + d2) * e3 + d3
// is sent to the element offset d0*s0 + d1*s1 + d2*s2 + d3*s3. Unused
// trailing dimensions have extent 1 and stride 0.
// --------------------------------------------------------------------------

struct IdxMap {
  int32_t e1, e2, e3;      // extents of dims 1..3 (dim 0 is implicit)
  int32_t pad_;
  int64_t s0, s1, s2, s3;  // strides in elements
};

inline IdxMap imap1(int64_t s0) { return IdxMap{1, 1, 1, 0, s0, 0, 0, 0}; }
inline IdxMap imap2(int32_t e1, int64_t s0, int64_t s1) {
  return IdxMap{e1, 1, 1, 0, s0, s1, 0, 0};
}
inline IdxMap imap3(int32_t e1, int32_t e2, int64_t s0, int64_t s1, int64_t s2) {
  return IdxMap{e1, e2, 1, 0, s0, s1, s2, 0};
}

__host__ __device__ inline int64_t imap_off(const IdxMap &m, int32_t x) {
  int32_t d3 = x % m.e3;
  x /= m.e3;
  int32_t d2 = x % m.e2;
  x /= m.e2;
  int32_t d1 = x % m.e1;
  int32_t d0 = x / m.e1;
  return d0 * m.s0 + d1 * m.s1 + d2 * m.s2 + d3 * m.s3;
}

// C(m, n) = alpha * sum_k A(m, k) B(k, n) + beta * C(m, n) on the matrix cores.
// Element (m, k) of A is A[imap_off(am, m) + imap_off(ak, k)], and so on.
// kfast_a: neighbouring k of A are adjacent in memory (else neighbouring m);
// nfast_b: neighbouring n of B are adjacent (else neighbouring k).
struct GemmDesc {
  int32_t M, N, K;
  const double *A;
  IdxMap am, ak;
  const double *B;
  IdxMap bk, bn;
  double *C;
  IdxMap cm, cn;
  double alpha, beta;
  bool kfast_a, nfast_b;
  int32_t prec;  // gxy_precision of the matrix-core arithmetic (0 = FP64)
};

void gemm(const GemmDesc &g, hipStream_t s);

// One dense sub-product of a grouped launch: M x N x K, tiles numbered from
// tile_start; ar/ac/br/bc/cr/cc index the shared int64 offset table.
struct GGroup {
  int32_t M, N, K, tile_start;
  int64_t ar, ac, br, bc, cr, cc;
};

// Output tile of a grouped launch: 64 (64 x 64), 128 (128 x 128) or 256
// (256 rows x 128 columns).
inline int tile_rows(int tile) { return tile; }
inline int tile_cols(int tile) { return tile == 256 ? 128 : tile; }

// Many independent sub-products in one launch (charge blocks), one output
// tile shape for every group of the launch. prec (gxy_precision) selects
// what the matrix cores compute in; operands and C stay FP64.
struct GroupedGemm {
  int32_t ngroups, total_tiles, tile, prec;
  const GGroup *groups;
  const int64_t *tab;
  const double *A, *B;
  double *C;
  double alpha, beta;
  bool kfast_a, nfast_b;
  // contig: every group's reduction and column indices are contiguous
  // ranges; its fields then read ar = row table (A and C rows), ac = A
  // column base, br = B base, bc = B row stride, cc = C column base, and
  // A(m, k) = A[tab[ar + m] + ac + k], B(k, n) = B[br + k bc + n],
  // C(m, n) = C[tab[ar + m] + cc + n]
  bool contig;
  // FP64 contiguous launches: stage operands by direct global -> LDS loads
  // (another summation order than the register-staged kernel)
  bool dma;
  // symmetric groups (C = A A^T, square tiles, beta = 0): tile t of a group
  // is (tm, tn) with tm >= tn in row-major triangular order, and each
  // off-diagonal tile also writes its transpose
  bool sym;
};

void grouped_gemm(const GroupedGemm &g, hipStream_t s);

// --------------------------------------------------------------------------
// configurational-temperature estimator, compact U(1) gauge theory (lgt.hip)
// --------------------------------------------------------------------------
// workspace (doubles) of one call; results: 14 doubles per configuration
size_t lgt_workspace_doubles(int d, const int32_t *dims, int64_t nconf, bool full);
// called on the stream right before and after the gradient kernel (the
// estimator's dominant launch), e.g. to time it with events
struct LgtHooks {
  void (*begin)(void *arg, hipStream_t s);
  void (*end)(void *arg, hipStream_t s);
  void *arg;
};
void lgt_estimate(const double *theta, int d, const int32_t *dims, int64_t nconf, bool full,
                  double *ws, double *dres, hipStream_t s, const LgtHooks *hooks = nullptr);
// raw register layout of one v_mfma_f64_16x16x4_f64 (a[64], b[64] -> out[256])
void launch_mfma_probe(const double *a, const double *b, double *out, hipStream_t s);
// kind 0: f32 16x16x4 (a[64], b[64]); kind 1: bf16 16x16x32 (a[512], b[512])
void launch_mfma_probe32(int kind, const float *a, const float *b, float *out,
                         hipStream_t s);

// --------------------------------------------------------------------------
// coefficients and initial tensors (FP64)
// --------------------------------------------------------------------------

// t[0..2nmax] for n = -nmax..nmax; q = harmonic of the second coupling.
void launch_char_coeffs(double beta, double delta, int q, int nmax, int nquad,
                        double *t, hipStream_t s);
// F, FM, FM1 for Q in [-qmax, qmax] (h1 couples to cos q theta, FM1 is the
// cos q theta impurity); zero_field selects the exact deltas.
void launch_field_factors(double beta, double h, double h1, int q, int qmax,
                          int lmax, bool zero_field, double *F, double *FM,
                          double *FM1, hipStream_t s);
// Zero-field factors of cos^2 theta and cos^2 q theta insertions, Q in
// [-qmax, qmax]: delta_{Q,0} / 2 + (delta_{Q,2k} + delta_{Q,-2k}) / 4.
void launch_square_factors(int q, int qmax, double *F2, double *F2q, hipStream_t s);
// T[l][r][u][d] = sqrt(t_l t_r t_u t_d) * F(n_u + n_r - n_d - n_l).
void launch_init_tensor(const double *t, const double *F, int nmax, double *T,
                        hipStream_t s);

// --------------------------------------------------------------------------
// element-wise, reductions, permutations (FP64)
// --------------------------------------------------------------------------

// partial[] <- blockwise sums of x^2; final: out[0] = sqrt(sum), out[1] = ln,
// out[2] = 1/norm. Deterministic (fixed tree, no atomics).
void launch_fro_norm(const double *x, int64_t n, double *partial,
                     double *out3, hipStream_t s);
// x[i] *= *scale (device scalar)
void launch_scale(double *x, int64_t n, const double *scale, hipStream_t s);
// out[c][d][a][b] = in[a][b][c][d] with dims (A, B, C, D) -> (C, D, A, B)
void launch_swap_pairs(const double *in, double *out, int A, int B, int C,
                       int D, hipStream_t s);
// out[a][c][b][d] = in[a][b][c][d]
void launch_swap_middle(const double *in, double *out, int A, int B, int C,
                        int D, hipStream_t s);
// out[P1 * W + P2] = in[l][r][u][d], (l, u) = pinv[P1], (r, d) = pinv[P2]
// with pinv[P] = h * Dv + v and W = Dh * Dv.
void launch_block_gather(const double *in, double *out, const int32_t *pinv, int Dh, int Dv,
                         hipStream_t s);
// out[0] += sum_{l,u} T[l][l][u][u] (out zeroed first)
void launch_trace(const double *T, int Dh, int Dv, double *out, hipStream_t s);
// fill
void launch_fill(double *x, int64_t n, double v, hipStream_t s);
void launch_fill_i32(int32_t *x, int64_t n, int32_t v, hipStream_t s);
void launch_identity(double *P, int n, hipStream_t s);

// --------------------------------------------------------------------------
// eigensolver: batched block-Jacobi on symmetric matrices padded to
// multiples of 32 rows.
// --------------------------------------------------------------------------

struct EigBatch {
  int32_t nmat;
  int32_t *d_npad;     // padded size per matrix
  int64_t *d_off;      // element offset of each matrix in A and V
  int32_t *d_pairbase; // first pair index of each matrix (size nmat+1)
  int32_t *d_pair_mat; // matrix of each pair
  int32_t total_pairs;
  int32_t max_nb;      // largest number of 16-row blocks
  double *A, *V, *Q;   // matrices, eigenvectors, 32x32 rotations per pair
  int32_t *d_flags;    // per matrix: 1 if a rotation was applied this sweep
  double *d_scale;     // per matrix: absolute threshold scale
  int32_t *d_rtl;      // per-update-tile descriptors
  int32_t n_update_tiles;
  int32_t *d_pair_rot; // per pair: 1 if its subproblem was rotated this round
};

// Gathers E[idx[i]][idx[j]] of every sector into the padded matrices;
// padding rows get -1 on the diagonal. V <- identity.
void launch_eig_gather(const double *E, int nfused, const int32_t *d_sec_idx,
                       const int32_t *d_sec_start, const int32_t *d_sec_n,
                       int nsec, const EigBatch &b, hipStream_t s);
// One outer round of block Jacobi for every matrix. A coupling a_pq is
// rotated if |a_pq| > rel_tol sqrt(|a_pp a_qq|) and (|a_pq| > abs_tol scale or
// |a_pq| > gap_tol |a_pp - a_qq|); each pair subproblem gets inner_sweeps
// cyclic sweeps.
void launch_eig_round(const EigBatch &b, int round, double abs_tol, double rel_tol,
                      double gap_tol, int inner_sweeps, hipStream_t s);
// per-matrix max |diagonal|, reduced to the batch maximum; flags <- 1
void launch_eig_scale(const EigBatch &b, hipStream_t s);
void launch_eig_identity(const EigBatch &b, double *V, hipStream_t s);
// y = a x over n elements
void launch_eig_scaled_copy(int64_t n, double a, const double *x, double *y, hipStream_t s);

// Tridiagonal path for sector matrices of at most kTriMaxN rows, in two
// stages. launch_tri_values: A (gathered padded matrices) is overwritten
// with the reflectors right of the diagonal and the decreasing eigenvalues
// on the diagonal; work (shaped like A) keeps d, e, tau and the eigenvalues;
// Y and X (shaped like A) are scratch; h_sec_n holds the nsec sector sizes
// on the host. With allow_multi the reduction shares each large matrix
// between several workgroups of one cooperative launch when the device can
// hold the whole grid at once (GXY_TRI_MULTI_MIN: smallest shared sector,
// rows) (GXY_TRI_MULTI=0 keeps one workgroup per
// matrix); callers that may run two such launches at once (batch workers)
// pass false, since two half-placed cooperative grids would wait on each
// other. launch_tri_vectors: the
// leading min(n, kmax) eigenvectors into V (row-major, column c = c-th
// largest), for the matrices of side *d_side (0: the first nsec, 1: the
// rest) or for all if d_side is null; Y is scratch.
constexpr int kTriMaxN = 2048;
constexpr int kTriMaxVecs = 128;   // eigenvectors formed per matrix
void launch_tri_values(int nmat, int nsec, const int *h_sec_n, const int32_t *d_sec_n,
                       const int32_t *d_npad, const int64_t *d_off, double *A, double *Y,
                       double *X, double *work, bool allow_multi, hipStream_t s);
void launch_tri_vectors(int nmat, int nsec, int maxn, const int32_t *d_sec_n,
                        const int32_t *d_npad, const int64_t *d_off, const double *A, double *V,
                        double *Y, const double *work, int kmax, const double *d_side,
                        hipStream_t s);

// --------------------------------------------------------------------------
// selection and projector
// --------------------------------------------------------------------------

struct SelectArgs {
  // both sides: sectors 0..nsec-1 are left, nsec..2nsec-1 right
  int32_t nsec;
  const int32_t *d_sec_label;  // [nsec]
  const int32_t *d_sec_n;      // [nsec]
  const int64_t *d_mat_off;    // [2 nsec] offsets of the padded matrices
  const int32_t *d_mat_npad;   // [2 nsec]
  const double *A;             // converged matrices (eigenvalues on diagonal)
  int32_t dcut;
  int32_t ncand;               // total candidates per side (sum of sec_n)
  double tie_rel, side_tol;
  // workspace
  double *d_lam;               // [2 * ncand]
  int32_t *d_cand_sec;         // [2 * ncand]
  int32_t *d_cand_rank;        // [2 * ncand]
  int32_t *d_cand_col;         // [2 * ncand] column in the padded matrix
  int32_t *d_taken;            // [2 * ncand]
  // outputs
  int32_t *d_pick_sec;         // [dcut] sector (0..nsec-1) of each new state
  int32_t *d_pick_col;         // [dcut] eigenvector column
  int32_t *d_pick_label;       // [dcut]
  double *d_diag;              // [8]: epsL, epsR, side, lam_max, gap, ties, trE
};

void launch_select(const SelectArgs &a, hipStream_t s);
// P[nfused x dcut] from the chosen side's eigenvectors.
void launch_build_projector(const double *V, const int64_t *d_mat_off,
                            const int32_t *d_mat_npad, const int32_t *d_sec_idx,
                            const int32_t *d_sec_start, const int32_t *d_sec_n,
                            const int32_t *d_pick_sec, const int32_t *d_pick_col,
                            const double *d_diag, int nsec, int nfused,
                            int dcut, double *P, hipStream_t s);

// final: res[0] = lnz, res[1] = <cos>, res[2] = <cos q>, res[3] = status,
// res[4..5] = <m^2> of both, res[6..7] = beta V (<m^2> - <m>^2) (NaN where a
// chain is absent); trk = traces of the cos, cos q, cos^2, cos^2 q chains
void launch_finish(const double *lnc, int nsteps, double beta, const double *tr,
                   const double *const trk[4], double *res, hipStream_t s);
void launch_observables(int npts, const double *beta, const double *lnz,
                        const double *mh, const double *mh1, double dbeta,
                        double dh, double dh1, double *out, hipStream_t s);

}  // namespace gxy
