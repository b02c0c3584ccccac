// Learned surrogate of the gXY thermodynamics: a 2 -> 128 -> 128 -> 4
// multilayer perceptron (SiLU after both hidden layers, linear output) that
// maps (beta, Delta) to (f, C_v, chi, chi_n), the observables of Ch. 3
// (free energy, specific heat, the two susceptibilities). Trained by
// full-batch Adam on the mean squared error of standardised targets; used to
// propose where along beta the C_v and chi maxima lie, so that the HOTRG
// runs that locate the transition lines can be spent there.
//
// Device work:
//  * Xavier-uniform initialisation from a counter-based SplitMix64 stream;
//  * target transform (logarithm of selected columns) and standardisation
//    (FP64 statistics, one workgroup, fixed reduction order);
//  * training in FP32: forward, loss, backward (chain rule), Adam; every
//    reduction in a fixed order, so a run is bitwise reproducible; one epoch
//    is captured once as a HIP graph and replayed;
//  * inference: FP32, or a fused kernel whose 128 x 128 layer runs on the
//    BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation);
//  * proposals: per Delta column of a candidate lattice, the maxima along
//    beta of the predicted C_v and chi, refined by the vertex of the
//    parabola through the three points around each maximum.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "ctx.h"
#include "internal.h"

namespace gxy {
namespace {

constexpr int kH = 128;                 // hidden width
constexpr int kIn = 2, kOut = 4;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kIn;
constexpr int kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kOut * kH;
constexpr int kNParam = kOffB3 + kOut;  // 17412
static_assert(kNParam == 17412, "parameter count");

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t k) {
  // output number k (0-based) of the SplitMix64 stream seeded with seed
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Xavier-uniform weights (limit sqrt(6 / (fan_in + fan_out))), zero biases.
// Weight draws are numbered through W1, W2, W3 in order.
__global__ void init_kernel(float *p, uint64_t seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNParam) return;
  int64_t draw = -1;
  double lim = 0.0;
  if (i < kOffB1) {
    draw = i;
    lim = sqrt(6.0 / (kIn + kH));
  } else if (i >= kOffW2 && i < kOffB2) {
    draw = (i - kOffW2) + kH * kIn;
    lim = sqrt(6.0 / (kH + kH));
  } else if (i >= kOffW3 && i < kOffB3) {
    draw = (i - kOffW3) + kH * kIn + kH * kH;
    lim = sqrt(6.0 / (kH + kOut));
  }
  if (draw < 0) {
    p[i] = 0.0f;
    return;
  }
  const double u = (double)(splitmix_at(seed, (uint64_t)draw) >> 11) * 0x1.0p-53;
  p[i] = (float)((2.0 * u - 1.0) * lim);
}

// Statistics and standardised copies of the training data. One workgroup;
// column statistics in FP64 with a fixed tree order.
constexpr int kPrepThreads = 256;
__global__ void prep_kernel(const double *x, const double *y, int n, uint32_t log_mask,
                            int standardize, double *scal, float *xs, float *ys) {
  __shared__ double red[kPrepThreads];
  __shared__ double mean_s[6], std_s[6];
  for (int c = 0; c < 6; ++c) {
    for (int pass = 0; pass < 2; ++pass) {
      double acc = 0.0;
      for (int s = threadIdx.x; s < n; s += kPrepThreads) {
        double v = c < 2 ? x[2 * s + c] : y[4 * s + (c - 2)];
        if (c >= 2 && ((log_mask >> (c - 2)) & 1)) v = log(v);
        if (pass == 1) v = (v - mean_s[c]) * (v - mean_s[c]);
        acc += v;
      }
      red[threadIdx.x] = acc;
      __syncthreads();
      for (int w = kPrepThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        if (pass == 0)
          mean_s[c] = standardize ? red[0] / n : 0.0;
        else
          std_s[c] = standardize ? sqrt(red[0] / n) : 1.0;
        if (pass == 1 && !(std_s[c] > 0.0)) std_s[c] = 1.0;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x < 6) {
    scal[threadIdx.x] = mean_s[threadIdx.x];
    scal[6 + threadIdx.x] = std_s[threadIdx.x];
  }
  for (int s = threadIdx.x; s < n; s += kPrepThreads) {
    for (int c = 0; c < 2; ++c) xs[2 * s + c] = (float)((x[2 * s + c] - mean_s[c]) / std_s[c]);
    for (int c = 0; c < 4; ++c) {
      double v = y[4 * s + c];
      if ((log_mask >> c) & 1) v = log(v);
      ys[4 * s + c] = (float)((v - mean_s[2 + c]) / std_s[2 + c]);
    }
  }
}

// out[s][o] = act(b[o] + sum_i W[o][i] in[s][i]); h keeps the pre-activation.
__global__ void fwd_kernel(const float *in, int I, const float *W, const float *b, int O, int n,
                           float *h, float *a, int act) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * O) return;
  const int s = t / O, o = t % O;
  float acc = b[o];
  const float *w = W + (int64_t)o * I;
  const float *x = in + (int64_t)s * I;
  for (int i = 0; i < I; ++i) acc = fmaf(w[i], x[i], acc);
  if (h) h[t] = acc;
  a[t] = act ? silu(acc) : acc;
}

// loss = mean (y - t)^2 over n x 4; dy = 2 (y - t) / (4 n). One workgroup.
constexpr int kLossThreads = 256;
__global__ void loss_kernel(const float *y, const float *t, int n, float *dy, float *loss_out,
                            float *hist, const int *step) {
  __shared__ float red[kLossThreads];
  const int m = 4 * n;
  const float inv = 1.0f / (float)m;
  float acc = 0.0f;
  for (int e = threadIdx.x; e < m; e += kLossThreads) {
    const float d = y[e] - t[e];
    dy[e] = 2.0f * d * inv;
    acc = fmaf(d, d, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kLossThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float l = red[0] * inv;
    loss_out[0] = l;
    if (hist) hist[*step] = l;
  }
}

// gW[o][i] = sum_s dh[s][o] a[s][i] for i < I, gb[o] = sum_s dh[s][o] (i = I).
__global__ void gradw_kernel(const float *dh, int O, const float *a, int I, int n, float *gW,
                             float *gb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= O * (I + 1)) return;
  const int o = t / (I + 1), i = t % (I + 1);
  float acc = 0.0f;
  if (i < I) {
    for (int s = 0; s < n; ++s) acc = fmaf(dh[(int64_t)s * O + o], a[(int64_t)s * I + i], acc);
    gW[(int64_t)o * I + i] = acc;
  } else {
    for (int s = 0; s < n; ++s) acc += dh[(int64_t)s * O + o];
    gb[o] = acc;
  }
}

// dh_prev[s][i] = (sum_o dh[s][o] W[o][i]) silu'(h_prev[s][i])
__global__ void back_kernel(const float *dh, int O, const float *W, int I, const float *hprev,
                            int n, float *dprev) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * I) return;
  const int s = t / I, i = t % I;
  float acc = 0.0f;
  for (int o = 0; o < O; ++o) acc = fmaf(dh[(int64_t)s * O + o], W[(int64_t)o * I + i], acc);
  dprev[t] = acc * dsilu(hprev[t]);
}

// Adam with bias correction; the update number is *step + 1.
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, const int *step,
                            float lr, float b1, float b2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNParam) return;
  const int t = *step + 1;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float c1 = (float)(1.0 - pow((double)b1, (double)t));
  const float c2 = (float)(1.0 - pow((double)b2, (double)t));
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void tick_kernel(int *step) { *step += 1; }
__global__ void zero_int_kernel(int *x) { *x = 0; }

__global__ void zero_kernel(float *x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0f;
}

// network output (standardised) -> physical units
__device__ __forceinline__ double to_physical(float v, int c, const double *scal,
                                              uint32_t log_mask) {
  double r = (double)v * scal[6 + 2 + c] + scal[2 + c];
  if ((log_mask >> c) & 1) r = exp(r);
  return r;
}

__global__ void standardize_x_kernel(const double *x, int n, const double *scal, float *xs) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * n) return;
  const int c = t & 1;
  xs[t] = (float)((x[t] - scal[c]) / scal[6 + c]);
}

__global__ void unstandardize_kernel(const float *ys, int n, const double *scal,
                                     uint32_t log_mask, double *y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;
  y[t] = to_physical(ys[t], t & 3, scal, log_mask);
}

// Fused inference, 64 samples per workgroup of 256 threads (4 waves):
// layer 1 in FP32, layer 2 on the BF16 matrix cores with FP32 accumulation
// (activations and W2 rounded to bfloat16), layer 3 in FP32.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
constexpr int kInfS = 64;
__global__ __launch_bounds__(256) void infer_bf16_kernel(const double *x, int n,
                                                         const float *p, const double *scal,
                                                         uint32_t log_mask, double *y) {
  __shared__ bf16x8_t w2s[kH][kH / 8 + 1];   // W2[o][k], 8 consecutive k per cell
  __shared__ bf16x8_t a1s[kInfS][kH / 8 + 1];
  __shared__ float a2s[kInfS][kH + 1];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * kInfS;
  for (int e = tid; e < kH * kH; e += 256) {
    const int o = e / kH, k = e % kH;
    ((__bf16 *)&w2s[o][k >> 3])[k & 7] = (__bf16)p[kOffW2 + e];
  }
  for (int e = tid; e < kInfS * kH; e += 256) {
    const int sl = e / kH, o = e % kH;
    const int s = s0 + sl;
    float v = 0.0f;
    if (s < n) {
      const float x0 = (float)((x[2 * s] - scal[0]) / scal[6]);
      const float x1 = (float)((x[2 * s + 1] - scal[1]) / scal[7]);
      v = silu(fmaf(p[kOffW1 + 2 * o + 1], x1, fmaf(p[kOffW1 + 2 * o], x0, p[kOffB1 + o])));
    }
    ((__bf16 *)&a1s[sl][o >> 3])[o & 7] = (__bf16)v;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  float4_t acc[kH / 16];
#pragma unroll
  for (int j = 0; j < kH / 16; ++j) acc[j] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < kH / 8; kc += 4) {
    const bf16x8_t av = a1s[wave * 16 + li][kc + lk];
#pragma unroll
    for (int j = 0; j < kH / 16; ++j) {
      const bf16x8_t bv = w2s[j * 16 + li][kc + lk];
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[j], 0, 0, 0);
    }
  }
  // accumulator register r of lane l: row 4 (l / 16) + r, column l % 16
#pragma unroll
  for (int j = 0; j < kH / 16; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int sl = wave * 16 + 4 * lk + r, o = j * 16 + li;
      a2s[sl][o] = silu(acc[j][r] + p[kOffB2 + o]);
    }
  __syncthreads();
  {
    const int sl = tid >> 2, c = tid & 3;
    const int s = s0 + sl;
    float v = p[kOffB3 + c];
    for (int k = 0; k < kH; ++k) v = fmaf(p[kOffW3 + c * kH + k], a2s[sl][k], v);
    if (s < n) y[4 * s + c] = to_physical(v, c, scal, log_mask);
  }
}

// Candidate lattice: point (j, i) = (beta_i, Delta_j), row-major over j.
__global__ void lattice_kernel(int nbeta, int ndelta, double blo, double bhi, double dlo,
                               double dhi, double *x) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbeta * ndelta) return;
  const int j = t / nbeta, i = t % nbeta;
  x[2 * t] = blo + (bhi - blo) * (double)i / (double)(nbeta - 1);
  x[2 * t + 1] = dlo + (dhi - dlo) * (double)j / (double)(ndelta - 1);
}

// One thread per (Delta column, proposal kind): kind 0 = maximum of column
// cv_col, kind 1 = maximum of column chi_col along beta. The first maximum
// wins ties; the parabola through it and its neighbours moves it by at most
// half a spacing; the jitter adds jitter * (2u - 1) / 2 spacings with u from
// the SplitMix64 stream (draw number 2 j + kind).
__global__ void propose_kernel(const double *y, int nbeta, int ndelta, int cv_col, int chi_col,
                               double blo, double bhi, double dlo, double dhi, uint64_t seed,
                               double jitter, double *out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * ndelta) return;
  const int j = t >> 1, kind = t & 1;
  const int col = kind == 0 ? cv_col : chi_col;
  const double *row = y + (int64_t)j * nbeta * 4;
  int best = 0;
  double bv = row[col];
  for (int i = 1; i < nbeta; ++i) {
    const double v = row[4 * i + col];
    if (v > bv) {
      bv = v;
      best = i;
    }
  }
  double off = 0.0;
  if (best > 0 && best < nbeta - 1) {
    const double ym = row[4 * (best - 1) + col], yp = row[4 * (best + 1) + col];
    const double den = ym - 2.0 * bv + yp;
    if (den < 0.0) off = fmin(0.5, fmax(-0.5, 0.5 * (ym - yp) / den));
  }
  const double u = (double)(splitmix_at(seed, (uint64_t)t) >> 11) * 0x1.0p-53;
  const double h = (bhi - blo) / (double)(nbeta - 1);
  double b = blo + h * ((double)best + off + jitter * (2.0 * u - 1.0) * 0.5);
  b = fmin(bhi, fmax(blo, b));
  out[2 * t] = b;
  out[2 * t + 1] = dlo + (dhi - dlo) * (double)j / (double)(ndelta - 1);
}

inline int blocks(int64_t n, int t = 256) { return (int)((n + t - 1) / t); }

}  // namespace
}  // namespace gxy

using namespace gxy;

struct gxy_mlp {
  gxy_ctx *ctx = nullptr;
  int device = 0;
  hipStream_t stream = nullptr;   // own stream (captured epochs), ordered after ctx->stream
  hipEvent_t ev = nullptr;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  int *step = nullptr;
  float *loss = nullptr;
  double *scal = nullptr;   // x mean[2], y mean[4], x std[2], y std[4]
  uint32_t log_mask = 0;
  // per-sample buffers, capacity cap samples
  int cap = 0;
  float *xs = nullptr, *ys = nullptr, *h1 = nullptr, *a1 = nullptr, *h2 = nullptr,
        *a2 = nullptr, *yo = nullptr, *dy = nullptr, *d2 = nullptr, *d1 = nullptr;
  double *xd = nullptr, *yd = nullptr;
  float *hist = nullptr;
  int hist_cap = 0;
  std::vector<void *> owned;
};

namespace gxy {
namespace {

template <class T>
T *mlp_alloc(gxy_mlp *m, int64_t n) {
  void *q = nullptr;
  const hipError_t e = hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) fail(GXY_ENOMEM, "surrogate device allocation failed");
  m->owned.push_back(q);
  return (T *)q;
}

void release(gxy_mlp *m, void *q) {
  if (!q) return;
  for (auto &o : m->owned)
    if (o == q) {
      (void)hipFree(o);
      o = nullptr;
    }
}

void ensure_cap(gxy_mlp *m, int n) {
  if (n <= m->cap) return;
  for (void *q : {(void *)m->xs, (void *)m->ys, (void *)m->h1, (void *)m->a1, (void *)m->h2,
                  (void *)m->a2, (void *)m->yo, (void *)m->dy, (void *)m->d2, (void *)m->d1,
                  (void *)m->xd, (void *)m->yd})
    release(m, q);
  const int c = std::max(n, 256);
  m->xs = mlp_alloc<float>(m, 2LL * c);
  m->ys = mlp_alloc<float>(m, 4LL * c);
  m->h1 = mlp_alloc<float>(m, (int64_t)kH * c);
  m->a1 = mlp_alloc<float>(m, (int64_t)kH * c);
  m->h2 = mlp_alloc<float>(m, (int64_t)kH * c);
  m->a2 = mlp_alloc<float>(m, (int64_t)kH * c);
  m->yo = mlp_alloc<float>(m, 4LL * c);
  m->dy = mlp_alloc<float>(m, 4LL * c);
  m->d2 = mlp_alloc<float>(m, (int64_t)kH * c);
  m->d1 = mlp_alloc<float>(m, (int64_t)kH * c);
  m->xd = mlp_alloc<double>(m, 2LL * c);
  m->yd = mlp_alloc<double>(m, 4LL * c);
  m->cap = c;
}

// forward pass on m->xs[0..n), then loss and gradient into m->g
void forward_backward(gxy_mlp *m, int n, bool with_hist, hipStream_t s) {
  float *p = m->p, *g = m->g;
  hipLaunchKernelGGL(fwd_kernel, dim3(blocks((int64_t)n * kH)), dim3(256), 0, s, m->xs, kIn,
                     p + kOffW1, p + kOffB1, kH, n, m->h1, m->a1, 1);
  hipLaunchKernelGGL(fwd_kernel, dim3(blocks((int64_t)n * kH)), dim3(256), 0, s, m->a1, kH,
                     p + kOffW2, p + kOffB2, kH, n, m->h2, m->a2, 1);
  hipLaunchKernelGGL(fwd_kernel, dim3(blocks((int64_t)n * kOut)), dim3(256), 0, s, m->a2, kH,
                     p + kOffW3, p + kOffB3, kOut, n, (float *)nullptr, m->yo, 0);
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(kLossThreads), 0, s, m->yo, m->ys, n, m->dy,
                     m->loss, with_hist ? m->hist : (float *)nullptr, (const int *)m->step);
  hipLaunchKernelGGL(gradw_kernel, dim3(blocks(kOut * (kH + 1))), dim3(256), 0, s, m->dy, kOut,
                     m->a2, kH, n, g + kOffW3, g + kOffB3);
  hipLaunchKernelGGL(back_kernel, dim3(blocks((int64_t)n * kH)), dim3(256), 0, s, m->dy, kOut,
                     p + kOffW3, kH, m->h2, n, m->d2);
  hipLaunchKernelGGL(gradw_kernel, dim3(blocks(kH * (kH + 1))), dim3(256), 0, s, m->d2, kH,
                     m->a1, kH, n, g + kOffW2, g + kOffB2);
  hipLaunchKernelGGL(back_kernel, dim3(blocks((int64_t)n * kH)), dim3(256), 0, s, m->d2, kH,
                     p + kOffW2, kH, m->h1, n, m->d1);
  hipLaunchKernelGGL(gradw_kernel, dim3(blocks(kH * (kIn + 1))), dim3(256), 0, s, m->d1, kH,
                     m->xs, kIn, n, g + kOffW1, g + kOffB1);
  GXY_CHECK_LAUNCH();
}

// The surrogate works on its own stream (a capture needs a stream of its
// own); each call first orders it after the work already on the context's.
hipStream_t begin(gxy_mlp *m) {
  GXY_HIP(hipEventRecord(m->ev, m->ctx->stream));
  GXY_HIP(hipStreamWaitEvent(m->stream, m->ev, 0));
  return m->stream;
}

void epoch(gxy_mlp *m, int n, const gxy_train_cfg &c, hipStream_t s) {
  forward_backward(m, n, true, s);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(kNParam)), dim3(256), 0, s, m->p, m->g, m->m,
                     m->v, (const int *)m->step, c.lr, c.beta1, c.beta2, c.eps);
  hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(1), 0, s, m->step);
  GXY_CHECK_LAUNCH();
}

}  // namespace
}  // namespace gxy

extern "C" {

gxy_status gxy_mlp_create(gxy_ctx *ctx, uint64_t seed, gxy_mlp **out) {
  if (!ctx || !out) return GXY_EINVAL;
  *out = nullptr;
  gxy_mlp *m = new (std::nothrow) gxy_mlp();
  if (!m) return GXY_ENOMEM;
  m->ctx = ctx;
  m->device = ctx->device;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  m->p = mlp_alloc<float>(m, kNParam);
  m->g = mlp_alloc<float>(m, kNParam);
  m->m = mlp_alloc<float>(m, kNParam);
  m->v = mlp_alloc<float>(m, kNParam);
  m->step = mlp_alloc<int>(m, 1);
  m->loss = mlp_alloc<float>(m, 1);
  m->scal = mlp_alloc<double>(m, 12);
  const double unit[12] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1};
  GXY_HIP(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
  GXY_HIP(hipEventCreateWithFlags(&m->ev, hipEventDisableTiming));
  hipStream_t s = begin(m);
  GXY_HIP(hipMemcpyAsync(m->scal, unit, sizeof(unit), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(init_kernel, dim3(blocks(kNParam)), dim3(256), 0, s, m->p, seed);
  GXY_CHECK_LAUNCH();
  GXY_HIP(hipStreamSynchronize(s));
  *out = m;
  return GXY_OK;
  }
  catch (...) {
    for (void *q : m->owned)
      if (q) (void)hipFree(q);
    if (m->ev) (void)hipEventDestroy(m->ev);
    if (m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
    ctx->last_error = "surrogate creation failed";
    return GXY_ENOMEM;
  }
}

gxy_status gxy_mlp_destroy(gxy_mlp *m) {
  if (!m) return GXY_OK;
  (void)hipSetDevice(m->device);
  (void)hipStreamSynchronize(m->stream);
  for (void *q : m->owned)
    if (q) (void)hipFree(q);
  (void)hipEventDestroy(m->ev);
  (void)hipStreamDestroy(m->stream);
  delete m;
  return GXY_OK;
}

gxy_status gxy_mlp_params(gxy_mlp *m, float *get, const float *set) {
  if (!m) return GXY_EINVAL;
  gxy_ctx *ctx = m->ctx;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  hipStream_t s = begin(m);
  if (set) GXY_HIP(hipMemcpyAsync(m->p, set, kNParam * sizeof(float), hipMemcpyHostToDevice, s));
  if (get) GXY_HIP(hipMemcpyAsync(get, m->p, kNParam * sizeof(float), hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_mlp_scaling(gxy_mlp *m, double *out12, uint32_t *log_mask) {
  if (!m || !out12) return GXY_EINVAL;
  gxy_ctx *ctx = m->ctx;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  hipStream_t s = begin(m);
  GXY_HIP(hipMemcpyAsync(out12, m->scal, 12 * sizeof(double), hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  if (log_mask) *log_mask = m->log_mask;
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_mlp_grad(gxy_mlp *m, const float *x, const float *y, int32_t n, float *grad,
                        float *loss) {
  if (!m || !x || !y || n <= 0 || !grad) return GXY_EINVAL;
  gxy_ctx *ctx = m->ctx;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  hipStream_t s = begin(m);
  ensure_cap(m, n);
  GXY_HIP(hipMemcpyAsync(m->xs, x, 2 * (size_t)n * sizeof(float), hipMemcpyHostToDevice, s));
  GXY_HIP(hipMemcpyAsync(m->ys, y, 4 * (size_t)n * sizeof(float), hipMemcpyHostToDevice, s));
  forward_backward(m, n, false, s);
  GXY_HIP(hipMemcpyAsync(grad, m->g, kNParam * sizeof(float), hipMemcpyDeviceToHost, s));
  if (loss) GXY_HIP(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_mlp_train(gxy_mlp *m, const double *x, const double *y, int32_t n,
                         const gxy_train_cfg *cfg, float *loss_hist) {
  if (!m || !x || !y || n <= 0 || !cfg || cfg->epochs < 0) return GXY_EINVAL;
  if (cfg->log_targets & ~15u) return GXY_EINVAL;
  gxy_ctx *ctx = m->ctx;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  hipStream_t s = begin(m);
  ensure_cap(m, n);
  if (cfg->epochs > m->hist_cap) {
    release(m, m->hist);
    m->hist = mlp_alloc<float>(m, cfg->epochs);
    m->hist_cap = cfg->epochs;
  }
  GXY_HIP(hipMemcpyAsync(m->xd, x, 2 * (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
  GXY_HIP(hipMemcpyAsync(m->yd, y, 4 * (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(prep_kernel, dim3(1), dim3(kPrepThreads), 0, s, m->xd, m->yd, n,
                     cfg->log_targets, cfg->standardize ? 1 : 0, m->scal, m->xs, m->ys);
  m->log_mask = cfg->log_targets;
  // fresh optimiser state
  hipLaunchKernelGGL(zero_kernel, dim3(blocks(kNParam)), dim3(256), 0, s, m->m, kNParam);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks(kNParam)), dim3(256), 0, s, m->v, kNParam);
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, m->step);
  GXY_CHECK_LAUNCH();
  if (cfg->epochs > 0) {
    // capture one epoch and replay it; every kernel reads the update number
    // from device memory, so the replays are identical launches
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GXY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      epoch(m, n, *cfg, s);
    } catch (...) {
      hipGraph_t dummy = nullptr;
      (void)hipStreamEndCapture(s, &dummy);
      if (dummy) (void)hipGraphDestroy(dummy);
      throw;
    }
    GXY_HIP(hipStreamEndCapture(s, &graph));
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      GXY_HIP(ie);
    }
    hipError_t le = hipSuccess;
    for (int e = 0; e < cfg->epochs && le == hipSuccess; ++e) le = hipGraphLaunch(exec, s);
    const hipError_t se = hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    GXY_HIP(le);
    GXY_HIP(se);
  }
  if (loss_hist && cfg->epochs > 0)
    GXY_HIP(hipMemcpyAsync(loss_hist, m->hist, cfg->epochs * sizeof(float),
                           hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_mlp_predict(gxy_mlp *m, const double *x, int32_t n, int32_t bf16, double *y) {
  if (!m || !x || n <= 0 || !y) return GXY_EINVAL;
  gxy_ctx *ctx = m->ctx;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  hipStream_t s = begin(m);
  ensure_cap(m, n);
  GXY_HIP(hipMemcpyAsync(m->xd, x, 2 * (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
  if (bf16) {
    hipLaunchKernelGGL(infer_bf16_kernel, dim3(blocks(n, kInfS)), dim3(256), 0, s, m->xd, n,
                       m->p, m->scal, m->log_mask, m->yd);
  } else {
    float *p = m->p;
    hipLaunchKernelGGL(standardize_x_kernel, dim3(blocks(2LL * n)), dim3(256), 0, s, m->xd, n,
                       m->scal, m->xs);
    hipLaunchKernelGGL(fwd_kernel, dim3(blocks((int64_t)n * kH)), dim3(256), 0, s, m->xs, kIn,
                       p + kOffW1, p + kOffB1, kH, n, (float *)nullptr, m->a1, 1);
    hipLaunchKernelGGL(fwd_kernel, dim3(blocks((int64_t)n * kH)), dim3(256), 0, s, m->a1, kH,
                       p + kOffW2, p + kOffB2, kH, n, (float *)nullptr, m->a2, 1);
    hipLaunchKernelGGL(fwd_kernel, dim3(blocks((int64_t)n * kOut)), dim3(256), 0, s, m->a2, kH,
                       p + kOffW3, p + kOffB3, kOut, n, (float *)nullptr, m->yo, 0);
    hipLaunchKernelGGL(unstandardize_kernel, dim3(blocks(4LL * n)), dim3(256), 0, s, m->yo, n,
                       m->scal, m->log_mask, m->yd);
  }
  GXY_CHECK_LAUNCH();
  GXY_HIP(hipMemcpyAsync(y, m->yd, 4 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  return GXY_OK;
  GXY_API_END(ctx)
}

gxy_status gxy_mlp_propose(gxy_mlp *m, const gxy_propose_cfg *c, double *beta_delta) {
  if (!m || !c || !beta_delta) return GXY_EINVAL;
  if (c->nbeta < 3 || c->ndelta < 2 || c->cv_col < 0 || c->cv_col > 3 || c->chi_col < 0 ||
      c->chi_col > 3 || !(c->beta_hi > c->beta_lo) || !(c->delta_hi > c->delta_lo) ||
      !(c->jitter >= 0.0 && c->jitter <= 1.0) ||
      (int64_t)c->nbeta * c->ndelta > (int64_t)1 << 26)
    return GXY_EINVAL;
  gxy_ctx *ctx = m->ctx;
  GXY_API_BEGIN
  GXY_HIP(hipSetDevice(ctx->device));
  hipStream_t s = begin(m);
  const int n = c->nbeta * c->ndelta;
  ensure_cap(m, n);
  hipLaunchKernelGGL(lattice_kernel, dim3(blocks(n)), dim3(256), 0, s, c->nbeta, c->ndelta,
                     c->beta_lo, c->beta_hi, c->delta_lo, c->delta_hi, m->xd);
  hipLaunchKernelGGL(infer_bf16_kernel, dim3(blocks(n, kInfS)), dim3(256), 0, s, m->xd, n,
                     m->p, m->scal, m->log_mask, m->yd);
  double *out = (double *)m->d1;  // 4 ndelta doubles, fits the d1 buffer (128 cap floats)
  hipLaunchKernelGGL(propose_kernel, dim3(blocks(2LL * c->ndelta)), dim3(256), 0, s, m->yd,
                     c->nbeta, c->ndelta, c->cv_col, c->chi_col, c->beta_lo, c->beta_hi,
                     c->delta_lo, c->delta_hi, c->seed, c->jitter, out);
  GXY_CHECK_LAUNCH();
  GXY_HIP(hipMemcpyAsync(beta_delta, out, 4 * (size_t)c->ndelta * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  GXY_HIP(hipStreamSynchronize(s));
  return GXY_OK;
  GXY_API_END(ctx)
}

}  // extern "C"
