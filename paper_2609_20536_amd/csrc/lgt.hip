// Configurational-temperature estimator for compact U(1) lattice gauge
// theory (Ch. 4, eq. another-form; Ch. 5, eqs. grad_hess and beta_lat):
// for a batch of link configurations theta_mu(n) on a periodic
// d-dimensional lattice (d = 2, 3, 4), the sums over links of g_l^2 and of
// h_ll, g^T h g, the plaquette average, and the estimators
// Tr h / |g|^2 (diagonal form, the thesis's four-dimensional one) and
// Tr h / |g|^2 - 2 g^T h g / |g|^4 (the divergence of g / |g|^2).
//
// g_l = sum over the 2(d - 1) plaquettes P of link l of s_{P,l} sin theta_P,
// h_ll = sum of cos theta_P over the same plaquettes, and
// g^T h g = sum over plaquettes of cos theta_P (sum_{l in P} s_{P,l} g_l)^2
// (the Hessian of the Wilson action is a sum of one rank-one term
// s s^T cos theta_P per plaquette), where s_{P,l} = +-1 is the sign of
// theta_l in theta_{mu nu}(n) = theta_mu(n) + theta_nu(n + mu) -
// theta_mu(n + nu) - theta_nu(n).
//
// Kernels (all FP64):
//  1. links: U = e^{i theta} once per link (one sincos each), so that every
//     plaquette is a product of four unit complex numbers, with no further
//     transcendental function;
//  2. grad: one thread per site; for each plane (a, b) it forms the site's
//     own plaquette and the two plaquettes based at n - b and n - a that
//     hold its a- and b-links, and so has every plaquette of its d links:
//     g, h, the per-direction sums and the site's plaquettes' cosines are
//     summed per workgroup (g is also written when g^T h g is asked for);
//  3. ghg: one thread per site, cos theta_P times the squared signed sum of
//     g over the links of each of the site's plaquettes;
//  4. reduce: one workgroup per configuration adds the workgroups' partial
//     sums in a fixed order and forms the estimators.
// Sites are x = x_0 + L_0 (x_1 + L_1 (x_2 + L_2 x_3)); links of direction mu
// of configuration c start at theta + (c d + mu) V.
#include <algorithm>

#include "internal.h"

namespace gxy {

namespace {

constexpr int kLgtThreads = 256;
constexpr int kLgtParts = 3 + 2 * 4;   // g2, h, plaquette, g2 per direction, h per direction

struct LgtGeom {
  int L[4];
  int st[4];           // st[mu] = L_0 ... L_{mu-1}
  int64_t V;
  int64_t nblk;        // site blocks per configuration
};

typedef double double2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2_t cmul(double2_t a, double2_t b) {
  return double2_t{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2_t cmulc(double2_t a, double2_t b) {   // a conj(b)
  return double2_t{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// U_a(n) U_b(n + a) conj(U_a(n + b)) conj(U_b(n)) = e^{i theta_ab(n)}
__device__ __forceinline__ double2_t plaq(double2_t ua, double2_t ub_a, double2_t ua_b,
                                          double2_t ub) {
  return cmulc(cmulc(cmul(ua, ub_a), ua_b), ub);
}

// Coordinates of one site; sites of a configuration fit int32 (the entry
// point refuses lattices of 2^31 sites or more), so neighbour indices are
// 32-bit.
template <int D>
struct Site {
  int x;
  int c[D];
  __device__ Site(const LgtGeom &G, int x_) : x(x_) {
    unsigned r = (unsigned)x_;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
      c[mu] = (int)(r % (unsigned)G.L[mu]);
      r /= (unsigned)G.L[mu];
    }
  }
  __device__ static int wrap(int cc, int L) { return cc < 0 ? cc + L : (cc >= L ? cc - L : cc); }
  // site index of x + k mu (k = +-1), periodic
  __device__ int nb(const LgtGeom &G, int mu, int k) const {
    return x + (wrap(c[mu] + k, G.L[mu]) - c[mu]) * G.st[mu];
  }
  // site index of x + k1 mu + k2 nu (mu != nu)
  __device__ int nb2(const LgtGeom &G, int mu, int k1, int nu, int k2) const {
    return x + (wrap(c[mu] + k1, G.L[mu]) - c[mu]) * G.st[mu] +
           (wrap(c[nu] + k2, G.L[nu]) - c[nu]) * G.st[nu];
  }
};

__global__ void lgt_links_kernel(const double *theta, double2_t *U, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s, c;
    sincos(theta[i], &s, &c);
    U[i] = double2_t{c, s};
  }
}

// Site block of this workgroup: workgroups go to the 8 XCDs in turn, so
// block b is renumbered to give each XCD (own L2) a contiguous band of sites,
// whose neighbours in the slowest directions then mostly sit in the same L2.
__device__ __forceinline__ int64_t lgt_block(int64_t nblk) {
  const int64_t b = blockIdx.x;
  return (nblk & 7) == 0 ? (b & 7) * (nblk >> 3) + (b >> 3) : b;
}

// sum of v over the workgroup into out (thread 0), fixed order
__device__ __forceinline__ double lgt_block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kLgtThreads / 64; ++w) t += red[w];
  return t;
}

template <int D>
__global__ __launch_bounds__(kLgtThreads) void lgt_grad_kernel(const double2_t *U, LgtGeom G,
                                                               int64_t nconf, double *gout,
                                                               double *partial) {
  __shared__ double red[kLgtThreads / 64];
  const int64_t cf = blockIdx.y;
  const int64_t blk = lgt_block(G.nblk);
  const int64_t x64 = blk * kLgtThreads + threadIdx.x;
  const bool act = x64 < G.V;
  const int x = (int)x64;
  const double2_t *Uc = U + cf * D * G.V;
  double g[D], h[D], pl = 0.0;
#pragma unroll
  for (int mu = 0; mu < D; ++mu) g[mu] = h[mu] = 0.0;
  if (act) {
    const Site<D> s(G, x);
    const double2_t *Ud[D];
    double2_t u[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
      Ud[mu] = Uc + mu * G.V;
      u[mu] = Ud[mu][x];
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = a + 1; b < D; ++b) {
        const double2_t *Ua = Ud[a], *Ub = Ud[b];
        // own plaquette theta_ab(x): link (x, a) with +, link (x, b) with -
        const double2_t p0 = plaq(u[a], Ub[s.nb(G, a, 1)], Ua[s.nb(G, b, 1)], u[b]);
        g[a] += p0.y;
        h[a] += p0.x;
        g[b] -= p0.y;
        h[b] += p0.x;
        pl += p0.x;
        // theta_ab(x - b): link (x, a) is its theta_a(n + b), with -
        const int yb = s.nb(G, b, -1);
        const double2_t p1 = plaq(Ua[yb], Ub[s.nb2(G, b, -1, a, 1)], u[a], Ub[yb]);
        g[a] -= p1.y;
        h[a] += p1.x;
        // theta_ab(x - a): link (x, b) is its theta_b(n + a), with +
        const int ya = s.nb(G, a, -1);
        const double2_t p2 = plaq(Ua[ya], u[b], Ua[s.nb2(G, a, -1, b, 1)], Ub[ya]);
        g[b] += p2.y;
        h[b] += p2.x;
      }
    if (gout) {
#pragma unroll
      for (int mu = 0; mu < D; ++mu) gout[(cf * D + mu) * G.V + x64] = g[mu];
    }
  }
  double vals[kLgtParts];
  double g2 = 0.0, hs = 0.0;
#pragma unroll
  for (int mu = 0; mu < D; ++mu) {
    g2 += g[mu] * g[mu];
    hs += h[mu];
  }
  vals[0] = g2;
  vals[1] = hs;
  vals[2] = pl;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) vals[3 + mu] = vals[7 + mu] = 0.0;
#pragma unroll
  for (int mu = 0; mu < D; ++mu) {
    vals[3 + mu] = g[mu] * g[mu];
    vals[7 + mu] = h[mu];
  }
  double *po = partial + (cf * G.nblk + blk) * (kLgtParts + 1);
#pragma unroll
  for (int k = 0; k < kLgtParts; ++k) {
    const double t = lgt_block_sum(vals[k], red);
    if (threadIdx.x == 0) po[k] = t;
  }
}

template <int D>
__global__ __launch_bounds__(kLgtThreads) void lgt_ghg_kernel(const double2_t *U, const double *g,
                                                              LgtGeom G, double *partial) {
  __shared__ double red[kLgtThreads / 64];
  const int64_t cf = blockIdx.y;
  const int64_t blk = lgt_block(G.nblk);
  const int64_t x64 = blk * kLgtThreads + threadIdx.x;
  double acc = 0.0;
  if (x64 < G.V) {
    const int x = (int)x64;
    const Site<D> s(G, x);
    const double2_t *Ud[D];
    const double *gd[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
      Ud[mu] = U + (cf * D + mu) * G.V;
      gd[mu] = g + (cf * D + mu) * G.V;
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = a + 1; b < D; ++b) {
        const int xa = s.nb(G, a, 1), xb = s.nb(G, b, 1);
        const double2_t p = plaq(Ud[a][x], Ud[b][xa], Ud[a][xb], Ud[b][x]);
        const double curl = gd[a][x] + gd[b][xa] - gd[a][xb] - gd[b][x];
        acc += p.x * curl * curl;
      }
  }
  const double t = lgt_block_sum(acc, red);
  if (threadIdx.x == 0) partial[(cf * G.nblk + blk) * (kLgtParts + 1) + kLgtParts] = t;
}

// out[c] = {sum_g2, sum_h, g_h_g, plaquette, beta_diag, beta_full,
//           sum_g2_dir[4], sum_h_dir[4]}
__global__ __launch_bounds__(kLgtThreads) void lgt_reduce_kernel(const double *partial,
                                                                 int64_t nblk, int d,
                                                                 int64_t nplaq, int full,
                                                                 double *out) {
  __shared__ double red[kLgtThreads / 64];
  const int64_t cf = blockIdx.x;
  const double *pc = partial + cf * nblk * (kLgtParts + 1);
  double tot[kLgtParts + 1];
  tot[kLgtParts] = 0.0;
  for (int k = 0; k < kLgtParts + full; ++k) {
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += kLgtThreads) v += pc[b * (kLgtParts + 1) + k];
    tot[k] = lgt_block_sum(v, red);
  }
  if (threadIdx.x == 0) {
    double *o = out + cf * 14;
    const double g2 = tot[0], hs = tot[1];
    o[0] = g2;
    o[1] = hs;
    o[2] = full ? tot[kLgtParts] : __builtin_nan("");
    o[3] = tot[2] / (double)nplaq;
    o[4] = hs / g2;
    o[5] = full ? hs / g2 - 2.0 * tot[kLgtParts] / (g2 * g2) : __builtin_nan("");
    for (int mu = 0; mu < 4; ++mu) {
      o[6 + mu] = mu < d ? tot[3 + mu] : 0.0;
      o[10 + mu] = mu < d ? tot[7 + mu] : 0.0;
    }
  }
}

template <int D>
void lgt_launch(const double *theta, const int32_t *dims, int64_t nconf, bool full, double *ws,
                double *dres, hipStream_t s, const LgtHooks *hooks) {
  LgtGeom G{};
  int64_t V = 1;
  for (int mu = 0; mu < 4; ++mu) {
    G.L[mu] = mu < D ? dims[mu] : 1;
    G.st[mu] = (int)V;
    if (mu < D) V *= dims[mu];
  }
  G.V = V;
  G.nblk = (V + kLgtThreads - 1) / kLgtThreads;
  const int64_t nlinks = nconf * D * V;
  double2_t *U = reinterpret_cast<double2_t *>(ws);
  double *g = full ? ws + 2 * nlinks : nullptr;
  double *partial = ws + (full ? 3 : 2) * nlinks;
  const int64_t lgrid = std::min<int64_t>((nlinks + kLgtThreads - 1) / kLgtThreads, 1 << 16);
  hipLaunchKernelGGL(lgt_links_kernel, dim3((unsigned)lgrid), dim3(kLgtThreads), 0, s, theta, U,
                     nlinks);
  GXY_CHECK_LAUNCH();
  const dim3 grid((unsigned)G.nblk, (unsigned)nconf);
  if (hooks) hooks->begin(hooks->arg, s);
  hipLaunchKernelGGL((lgt_grad_kernel<D>), grid, dim3(kLgtThreads), 0, s, U, G, nconf, g,
                     partial);
  GXY_CHECK_LAUNCH();
  if (hooks) hooks->end(hooks->arg, s);
  if (full) {
    hipLaunchKernelGGL((lgt_ghg_kernel<D>), grid, dim3(kLgtThreads), 0, s, U, g, G, partial);
    GXY_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(lgt_reduce_kernel, dim3((unsigned)nconf), dim3(kLgtThreads), 0, s, partial,
                     G.nblk, D, V * (D * (D - 1) / 2), full ? 1 : 0, dres);
  GXY_CHECK_LAUNCH();
}

}  // namespace

size_t lgt_workspace_doubles(int d, const int32_t *dims, int64_t nconf, bool full) {
  int64_t V = 1;
  for (int mu = 0; mu < d; ++mu) V *= dims[mu];
  const int64_t nlinks = nconf * d * V;
  const int64_t nblk = (V + kLgtThreads - 1) / kLgtThreads;
  return (size_t)((full ? 3 : 2) * nlinks + nconf * nblk * (kLgtParts + 1) + nconf * 14);
}

void lgt_estimate(const double *theta, int d, const int32_t *dims, int64_t nconf, bool full,
                  double *ws, double *dres, hipStream_t s, const LgtHooks *hooks) {
  switch (d) {
    case 2: lgt_launch<2>(theta, dims, nconf, full, ws, dres, s, hooks); break;
    case 3: lgt_launch<3>(theta, dims, nconf, full, ws, dres, s, hooks); break;
    case 4: lgt_launch<4>(theta, dims, nconf, full, ws, dres, s, hooks); break;
    default: fail(GXY_EINVAL, "lattice dimension must be 2, 3 or 4");
  }
}

}  // namespace gxy
