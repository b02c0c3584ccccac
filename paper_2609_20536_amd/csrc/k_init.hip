// Character coefficients, field factors and initial site tensors (FP64).
//
// t_n = (1/Q) sum_k w(phi_k) cos(n phi_k), phi_k = 2 pi k / Q, with
// w(phi) = exp(beta [Delta cos phi + (1 - Delta) cos q phi]): the character
// coefficient a_n(beta, Delta) of Ch. 3 (eq. a_n) written as the Fourier
// integral of the bond weight and evaluated by the periodic trapezoid rule.
// The Hamiltonian (Ch. 3, eq. gXY_ham) has a general harmonic q; the thesis
// takes q = 2. Site tensor (Ch. 3, final site-tensor equation):
//   T[l][r][u][d] = sqrt(t_l t_r t_u t_d) * F(n_u + n_r - n_d - n_l),
//   F(Q) = sum_l I_{Q+ql}(beta h) I_l(beta h1)   (h1 couples to cos q theta),
// and the impurity tensors with F_M (cos theta), F_M1 (cos q theta) (Ch. 3,
// the two impure-tensor equations).
#include "internal.h"

namespace gxy {

namespace {

constexpr int kCoeffThreads = 256;

__global__ void char_coeffs_kernel(double beta, double delta, int q, int nmax,
                                   int nquad, double *t) {
  __shared__ double red[kCoeffThreads];
  const int n = blockIdx.x;  // 0..nmax
  double acc = 0.0;
  for (int k = threadIdx.x; k < nquad; k += kCoeffThreads) {
    double phi = 2.0 * M_PI * (double)k / (double)nquad;
    double w = exp(beta * (delta * cos(phi) + (1.0 - delta) * cos((double)q * phi)));
    acc += w * cos((double)n * phi);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kCoeffThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double v = red[0] / (double)nquad;
    v = v > 0.0 ? v : 0.0;  // exact coefficients are non-negative
    t[nmax + n] = v;
    t[nmax - n] = v;        // t_{-n} = t_n since w is even
  }
}

// I_k(x) by its power series sum_j (x/2)^(2j+k) / (j! (j+k)!), I_{-k} = I_k.
__device__ double bessel_i(int k, double x) {
  k = k < 0 ? -k : k;
  if (x == 0.0) return k == 0 ? 1.0 : 0.0;
  const double half = 0.5 * x;
  double term = 1.0;
  for (int j = 1; j <= k; ++j) term *= half / (double)j;
  double total = term;
  for (int j = 1; j < 400; ++j) {
    term *= half * half / ((double)j * (double)(j + k));
    total += term;
    if (term <= 1e-18 * total) break;
  }
  return total;
}

__global__ void field_factors_kernel(double beta, double h, double h1, int q, int qmax,
                                     int lmax, int zero_field, double *F,
                                     double *FM, double *FM1) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a > 2 * qmax) return;
  const int Q = a - qmax;
  if (zero_field) {
    F[a] = Q == 0 ? 1.0 : 0.0;
    FM[a] = (Q == 1 || Q == -1) ? 0.5 : 0.0;
    FM1[a] = (Q == q || Q == -q) ? 0.5 : 0.0;
    return;
  }
  const double x = beta * h, x1 = beta * h1;
  double f = 0.0, fm = 0.0, fm1 = 0.0;
  for (int l = -lmax; l <= lmax; ++l) {
    const double il1 = bessel_i(l, x1);
    const double iq = bessel_i(Q + q * l, x);
    f += iq * il1;
    fm += il1 * 0.5 * (bessel_i(Q + q * l - 1, x) + bessel_i(Q + q * l + 1, x));
    fm1 += iq * 0.5 * (bessel_i(l + 1, x1) + bessel_i(l - 1, x1));
  }
  F[a] = f;
  FM[a] = fm;
  FM1[a] = fm1;
}

__global__ void init_tensor_kernel(const double *t, const double *F, int nmax,
                                   double *T) {
  const int D = 2 * nmax + 1;
  const int64_t total = (int64_t)D * D * D * D;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int d = (int)(e % D);
  const int u = (int)((e / D) % D);
  const int r = (int)((e / ((int64_t)D * D)) % D);
  const int l = (int)(e / ((int64_t)D * D * D));
  // charges n = index - nmax
  const int Q = (u - nmax) + (r - nmax) - (d - nmax) - (l - nmax);
  const double amp = sqrt(t[l] * t[r] * t[u] * t[d]);
  T[e] = amp * F[Q + 4 * nmax];
}

}  // namespace

void launch_char_coeffs(double beta, double delta, int q, int nmax, int nquad,
                        double *t, hipStream_t s) {
  hipLaunchKernelGGL(char_coeffs_kernel, dim3(nmax + 1), dim3(kCoeffThreads), 0,
                     s, beta, delta, q, nmax, nquad, t);
  GXY_CHECK_LAUNCH();
}

void launch_field_factors(double beta, double h, double h1, int q, int qmax, int lmax,
                          bool zero_field, double *F, double *FM, double *FM1,
                          hipStream_t s) {
  const int n = 2 * qmax + 1;
  hipLaunchKernelGGL(field_factors_kernel, dim3((n + 63) / 64), dim3(64), 0, s,
                     beta, h, h1, q, qmax, lmax, zero_field ? 1 : 0, F, FM, FM1);
  GXY_CHECK_LAUNCH();
}

// The site angle's integral of cos^2(k theta) e^{-i Q theta} / 2 pi, the
// factor of a site tensor with that insertion at zero field, k = 1 and q.
__global__ void square_factors_kernel(int q, int qmax, double *F2, double *F2q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > 2 * qmax) return;
  const int Q = i - qmax;
  const int aq = Q < 0 ? -Q : Q;
  F2[i] = (Q == 0 ? 0.5 : 0.0) + (aq == 2 ? 0.25 : 0.0);
  F2q[i] = (Q == 0 ? 0.5 : 0.0) + (aq == 2 * q ? 0.25 : 0.0);
}

void launch_square_factors(int q, int qmax, double *F2, double *F2q, hipStream_t s) {
  const int n = 2 * qmax + 1;
  hipLaunchKernelGGL(square_factors_kernel, dim3((n + 63) / 64), dim3(64), 0, s, q, qmax, F2,
                     F2q);
  GXY_CHECK_LAUNCH();
}

void launch_init_tensor(const double *t, const double *F, int nmax, double *T,
                        hipStream_t s) {
  const int D = 2 * nmax + 1;
  const int64_t total = (int64_t)D * D * D * D;
  hipLaunchKernelGGL(init_tensor_kernel, dim3((unsigned)((total + 255) / 256)),
                     dim3(256), 0, s, t, F, nmax, T);
  GXY_CHECK_LAUNCH();
}

}  // namespace gxy
