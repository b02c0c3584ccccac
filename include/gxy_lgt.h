/*
 * gxy_lgt.h — C ABI of the configurational-temperature estimator for compact
 * U(1) lattice gauge theory (Ch. 4 and 5 of the thesis), in the same
 * library and on the same contexts as gxy_hotrg.h.
 *
 * Model (Ch. 5, introduction): link angles theta_mu(n) on a periodic
 * d-dimensional lattice, the plaquette angle
 *   theta_{mu nu}(n) = theta_mu(n) + theta_nu(n + mu) - theta_mu(n + nu)
 *                      - theta_nu(n)            (mu < nu),
 * and the Wilson action S = beta sum_{n, mu < nu} (1 - cos theta_{mu nu}(n)).
 * With g_l = (1/beta) dS/dtheta_l and h_lm = (1/beta) d^2 S/dtheta_l
 * dtheta_m (Ch. 5, eq. grad_hess), the estimator of the coupling is the
 * divergence of g / |g|^2 (Ch. 4, eq. another-form; Ch. 5, eq. beta_lat):
 *   beta_full = Tr h / |g|^2 - 2 g^T h g / |g|^4,
 * and its diagonal form, which drops the Hessian's off-diagonal part as the
 * thesis does for four dimensions (Ch. 5, Sec. "Four-Dimensional Theory"):
 *   beta_diag = Tr h / |g|^2.
 * For configurations drawn from exp(-S) at coupling beta both estimate
 * beta; beta_full is the one the derivation gives, beta_diag and the
 * per-direction sums (Ch. 5, Sec. "Two-Dimensional Theory", beta_x) its
 * large-volume forms.
 */
#ifndef GXY_LGT_H
#define GXY_LGT_H

#include "gxy_hotrg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Flags of gxy_lgt_estimator. */
enum { GXY_LGT_FULL = 1u /* also g^T h g and beta_full */ };

/* Largest batch of one call (configurations). */
#define GXY_LGT_MAX_CONF 65535

/* Results for one configuration. Sums run over all links (l = (n, mu)) or
 * all plaquettes of the configuration. */
typedef struct {
  double sum_g2;         /* sum_l g_l^2                                      */
  double sum_h;          /* sum_l h_ll = Tr h                                 */
  double g_h_g;          /* g^T h g (NaN without GXY_LGT_FULL)               */
  double plaquette;      /* mean of cos theta_{mu nu}(n) over plaquettes      */
  double beta_diag;      /* sum_h / sum_g2 (IEEE: |g| = 0 gives inf or NaN)  */
  double beta_full;      /* sum_h/sum_g2 - 2 g_h_g/sum_g2^2 (NaN w/o FULL)    */
  double sum_g2_dir[4];  /* sum of g_l^2 over the links of direction mu       */
  double sum_h_dir[4];   /* sum of h_ll over the links of direction mu
                            (entries mu >= ndim are 0)                       */
} gxy_lgt_result;

/* Device workspace (bytes) that gxy_lgt_estimator needs for these
 * arguments (same validation; host only), for callers that supply it with
 * gxy_set_workspace. */
gxy_status gxy_lgt_workspace_bytes(int32_t ndim, const int32_t *dims, int64_t nconf,
                                   uint32_t flags, size_t *out);

/* The estimator for nconf configurations, in one pass over the batch on the
 * context's stream (synchronous: returns when out is filled).
 *   theta  device pointer, FP64 link angles (any real value; the estimator is
 *          periodic in each), layout theta[c][mu][x] with the site index
 *          x = x_0 + L_0 (x_1 + L_1 (x_2 + L_2 x_3)), c < nconf, mu < ndim;
 *          read only, owned by the caller, not retained
 *   ndim   2, 3 or 4
 *   dims   host array of ndim extents L_0..L_{ndim-1}, each >= 2 (periodic;
 *          a plaquette needs four distinct links)
 *   nconf  0..GXY_LGT_MAX_CONF (0: nothing to do)
 *   flags  0 or GXY_LGT_FULL
 *   out    host array of nconf results
 * Workspace: 16 bytes per link (U = e^{i theta}), 8 more per link with
 * GXY_LGT_FULL (g), and the partial sums, from the context's workspace.
 * Errors: GXY_EINVAL for a null context or pointer, ndim outside 2..4, an
 * extent below 2, more than 2^31 - 1 sites, nconf outside 0..
 * GXY_LGT_MAX_CONF or an unknown flag (no device work issued);
 * GXY_ENOMEM if the workspace cannot be had; GXY_EDEVICE for HIP errors. */
gxy_status gxy_lgt_estimator(gxy_ctx *ctx, const double *theta, int32_t ndim,
                             const int32_t *dims, int64_t nconf, uint32_t flags,
                             gxy_lgt_result *out);

#ifdef __cplusplus
}
#endif

#endif /* GXY_LGT_H */
