/*
 * gxy_hotrg_testing.h — entry points that expose single kernels of
 * libgxyhotrg for unit tests. They are not part of a HOTRG run's interface.
 * Host arrays are caller-owned; each call copies them to the device, runs the
 * kernel on the context's stream, copies the result back and synchronises.
 */
#ifndef GXY_HOTRG_TESTING_H
#define GXY_HOTRG_TESTING_H

#include "gxy_hotrg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C = A B with the FP64 MFMA GEMM of the contractions (the kernel behind the
 * environment and projection products of Ch. 2, eqs. hosvd and
 * renormalizedT). A is M x K (row-major, or stored as K x M if a_trans),
 * B is K x N (row-major, or stored as N x K if b_trans), C is M x N
 * row-major. a_trans/b_trans select the operand orientations the kernel
 * supports (reduction index adjacent or output index adjacent in memory). */
gxy_status gxy_test_gemm_f64(gxy_ctx *ctx, int32_t M, int32_t N, int32_t K,
                             const double *A, int32_t a_trans, const double *B,
                             int32_t b_trans, double *C);

/* The same product in one of the contraction forms (gxy_precision): FP64;
 * FP32 (operands rounded to FP32, FP32 accumulation); BF16X3 (operands
 * rounded to FP32 and split into bfloat16 hi + lo, hi*hi + hi*lo + lo*hi,
 * FP32 accumulation). Operands and C are FP64 in memory in every form. */
gxy_status gxy_test_gemm(gxy_ctx *ctx, int32_t prec, int32_t M, int32_t N, int32_t K,
                         const double *A, int32_t a_trans, const double *B,
                         int32_t b_trans, double *C);

/* Eigendecomposition of one symmetric n x n matrix (row-major) with the
 * batched block-Jacobi solver used for the environment matrices (Ch. 2,
 * eq. hosvd). w[n] receives the eigenvalues, V[n x n] (row-major) the
 * eigenvectors as columns, in the solver's (unsorted) order; *sweeps (may be
 * NULL) the number of block-Jacobi sweeps used. */
gxy_status gxy_test_eigh(gxy_ctx *ctx, int32_t n, const double *A, double *w,
                         double *V, int32_t *sweeps);

/* The same with the solver chosen: method 0 = as a run would, 1 = block
 * Jacobi, 2 = Householder tridiagonalisation + bisection + inverse
 * iteration (n <= 128 here, since all n eigenvectors are asked for; larger
 * n use block Jacobi). Eigenvalues w in the solver's column order. */
gxy_status gxy_test_eigh_method(gxy_ctx *ctx, int32_t method, int32_t n, const double *A,
                                double *w, double *V, int32_t *sweeps);

/* As a run needs it: every eigenvalue, and eigenvectors for (at least) the
 * kmax largest ones (1 <= kmax <= n). The tridiagonal path (n <= 1024,
 * kmax <= 128) returns eigenvalues in decreasing order with the leading
 * kmax columns of V filled (the rest zero); block Jacobi fills all. */
gxy_status gxy_test_eigh_top(gxy_ctx *ctx, int32_t method, int32_t n, int32_t kmax,
                             const double *A, double *w, double *V, int32_t *sweeps);

/* Register layout of one FP64 16x16x4 matrix-core instruction: lane l
 * supplies a[l] and b[l]; out[4 l + r] receives accumulator register r of
 * lane l (accumulator initially zero). */
gxy_status gxy_test_mfma_layout(gxy_ctx *ctx, const double *a, const double *b,
                                double *out);

/* Register layout of the FP32-accumulating matrix-core instructions used by
 * the reduced-precision contractions: kind 0 = 16x16x4 FP32 (a[64], b[64],
 * one value per lane), kind 1 = 16x16x32 BF16 (a[512], b[512], eight values
 * per lane, rounded to bfloat16 on the device). out[4 l + r] = accumulator
 * register r of lane l. */
gxy_status gxy_test_mfma_layout32(gxy_ctx *ctx, int32_t kind, const float *a,
                                  const float *b, float *out);

#ifdef __cplusplus
}
#endif

#endif
