/*
 * gxy_hotrg.h — C ABI of the MI355X (gfx950) HOTRG library for the 2D
 * generalized XY model.
 *
 * A run follows the thesis's statement of the problem (Ch. 3, "Tensor
 * Formulation" and "Derivation of Tensors for the Generalized XY Model";
 * Ch. 2, "Higher-Order Tensor Renormalization Group Method"):
 *   character coefficients t_n of exp(beta[Delta cos phi + (1-Delta) cos 2phi])
 *   -> rank-4 site tensor T[l][r][u][d] (and impurity tensors for <cos theta>,
 *      <cos 2 theta>)
 *   -> nsteps HOTRG coarse-graining steps (fused two-site tensor M, environment
 *      Gram matrices, FP64 eigendecomposition = HOSVD factors, truncation to
 *      dcut, projection P^T M P), alternating vertical / horizontal
 *   -> ln Z per site and the impurity expectation values.
 *
 * Conventions
 *   - Site tensor legs are (l, r, u, d); the charge law at zero field is
 *     q_l + q_d = q_r + q_u (the thesis's n1 + n2 - n3 - n4 = 0 with legs
 *     (top, right, bottom, left) = (u, r, d, l)).
 *   - Step 1 contracts the vertical bond; steps alternate.
 *   - All functions return a gxy_status; none aborts, exits or throws.
 *   - Host pointers are owned by the caller and only read/written during
 *     the call. Device memory is either library-allocated (hipMalloc, freed
 *     by gxy_destroy) or supplied by the caller through gxy_set_workspace.
 *   - Work is issued on the stream given to gxy_create; every call that
 *     returns results to host memory synchronises that stream before
 *     returning. One context must not be used by two host threads at once.
 *   - Nothing is printed unless the environment variable GXY_LOG is set.
 *   - A run uses two more streams of its own: one for the copies of the
 *     projection's offset tables and, for charge-block runs with impurity
 *     chains whose projection fits one chunk, one for the impurity
 *     projections of step n, which overlap the environments and eigensolves
 *     of step n + 1 (events order them; results are the same bits either
 *     way).
 *
 * Environment variables (read at each run unless noted)
 *   GXY_LOG                log error messages to stderr
 *   GXY_CHUNK_BYTES        bound of the projection's three D^5 buffers
 *                          (default 32 GiB; batch workers 4 GiB)
 *   GXY_NO_OVERLAP         keep the impurity projections on the main stream
 *   GXY_EIG                jacobi | tri: force one sector eigensolver
 *   GXY_JACOBI_MAX_SWEEPS  sweep limit of block Jacobi (default 120)
 *   GXY_TRI_MULTI          0: one workgroup per sector in the tridiagonal
 *                          reduction
 *   GXY_TRI_MULTI_MIN      smallest sector (rows) shared between workgroups
 *                          (default 384)
 *   GXY_TRI_COOP           0: launch the shared reduction as a regular grid
 *                          instead of a cooperative one (same results and
 *                          speed; for profilers that fail on cooperative
 *                          launches)
 *   GXY_PROJ_TILE          64 | 128 | 256: projection tile for every run
 *                          (else the autotuned one for the Dcut, else by
 *                          tile fill); results do not depend on it
 *   GXY_GEMM_DMA           1: the FP64 projection products stage their
 *                          operands by direct global -> LDS loads (faster
 *                          products, another summation order: results agree
 *                          with the default to rounding, and across tiles
 *                          bit for bit)
 *   GXY_BATCH_WORKERS      default worker count of gxy_run_batch (4)
 *   GXY_TIMING             phase timers (gxy_phase_times)
 *   GXY_INJECT_NAN_STEP    test hook of the failure path: one NaN is put into
 *                          the site tensor after step n's normalisation
 *   GXY_HOT_EVENTS         events around every launch of the D^7 product
 *                          (gxy_hot_kernel_stats)
 */
#ifndef GXY_HOTRG_H
#define GXY_HOTRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GXY_OK = 0,
  GXY_EINVAL = 1,        /* invalid argument; no device work was issued     */
  GXY_ENOMEM = 2,        /* device memory (or the caller's workspace) short */
  GXY_EDEVICE = 3,       /* a HIP runtime call failed                       */
  GXY_ENUMERIC = 4,      /* non-finite or non-positive trace, no eigen
                            convergence                                      */
  GXY_EUNSUPPORTED = 5,  /* valid request the library does not implement    */
  GXY_EPARTIAL = 6       /* batch: at least one run failed (see per-run)    */
} gxy_status;

/* Arithmetic of the projection contractions (the D^7 work of eq.
 * renormalizedT and the impurity placements). Tensors stay FP64 in memory;
 * the environments (eq. hosvd), their eigendecompositions, t_n, the norms
 * and the log-norm accumulation are FP64 in every form. */
typedef enum {
  GXY_PREC_FP64 = 0,     /* FP64 MFMA                                       */
  GXY_PREC_FP32 = 1,     /* operands rounded to FP32, FP32 MFMA, FP32
                            accumulation                                    */
  GXY_PREC_BF16X3 = 2    /* operands rounded to FP32, split x = hi + lo into
                            bfloat16 terms, hi*hi + hi*lo + lo*hi by BF16
                            MFMA with FP32 accumulation                     */
} gxy_precision;

/* Impurity chains. COS1 / COS2: one cos theta / cos q theta insertion
 * averaged over the sites (Ch. 3, the impure-tensor method). COS1_SQ /
 * COS2_SQ (zero field only): also two insertions averaged over ordered
 * pairs of sites, giving <m^2> and the susceptibility
 * beta V (<m^2> - <m>^2) of Ch. 3, eq. susc, from one run (a variant of the
 * impurity method the thesis does not use); each implies its first moment. */
enum { GXY_IMP_COS1 = 1u, GXY_IMP_COS2 = 2u, GXY_IMP_COS1_SQ = 4u, GXY_IMP_COS2_SQ = 8u };

/* One HOTRG run (one point of the (beta, Delta, h, h1) parameter space). */
typedef struct {
  double beta;          /* inverse temperature, >= 0                         */
  double delta;         /* deformation, 0 <= delta <= 1 (J = delta, J1 = 1-delta) */
  double h;             /* field coupling to cos theta                       */
  double h1;            /* field coupling to cos q theta                     */
  int32_t nmax;         /* charges |n| <= nmax, initial bond D0 = 2 nmax + 1; 0..64 */
  int32_t dcut;         /* truncation bond dimension, 1..128                 */
  int32_t nsteps;       /* coarse-graining steps, 0..62 (lattice 2^nsteps sites) */
  int32_t nquad;        /* quadrature points for t_n, > 2 nmax              */
  uint32_t impurities;  /* GXY_IMP_* bitmask                                 */
  int32_t prec;         /* gxy_precision of the projection contractions      */
  int32_t fp64_steps;   /* precision schedule: steps 1..fp64_steps contract in
                           FP64, later steps in prec (>= 0; step n enters
                           ln Z / N with weight 2^-n)                         */
  int32_t q;            /* harmonic of the second coupling, (1 - delta)
                           cos(q (theta_j - theta_k)) (Ch. 3, eq. gXY_ham;
                           the thesis studies q = 2), of the field h1 and of
                           the second impurity; 0 means 2; 2..16. At h = 0 !=
                           h1 the sectors are charge mod q                   */
} gxy_point;

typedef struct {
  double lnz_per_site;  /* ln Z / 2^nsteps                                   */
  double m_cos1;        /* <cos theta>   (NaN if not requested)              */
  double m_cos2;        /* <cos q theta> (NaN if not requested)              */
  double max_trunc_err; /* max over steps of eps_chosen / trace(E)          */
  double min_cut_gap;   /* min over steps of (lam_D - lam_{D+1}) / lam_1     */
  int32_t near_ties;    /* number of tie-rule activations                   */
  int32_t status;       /* gxy_status of this run                            */
  int32_t fail_step;    /* -1 if none; GXY_ENUMERIC: the step whose
                           environments or norm were first not finite, or
                           nsteps if only the final trace failed            */
  int32_t nsteps_done;
  double msq_cos1;      /* <m^2>, m = (1/V) sum_i cos theta_i (GXY_IMP_COS1_SQ;
                           else NaN); V = 2^nsteps                          */
  double msq_cos2;      /* the same for cos q theta (GXY_IMP_COS2_SQ)        */
  double chi0;          /* beta V (<m^2> - <m>^2) for cos theta: the
                           susceptibility at this (zero) field               */
  double chi0_n;        /* the same for cos q theta                          */
} gxy_result;

/* Per-step diagnostics of the last run (or of run `run` of the last batch). */
typedef struct {
  double lnc;           /* ln of the Frobenius norm divided out this step    */
  double eps_l, eps_r;  /* discarded weights of the left / right environment */
  double lam_max;       /* largest environment eigenvalue                    */
  double cut_gap;       /* (lam_D - lam_{D+1}) / lam_1 of the chosen side    */
  int32_t side;         /* 0 = left factor U, 1 = right factor V             */
  int32_t dh, dv;       /* bond dimensions after the step (l/r, u/d)         */
  int32_t truncated;    /* 0 if the fused bond fit (P = identity)            */
  int32_t ties;
  int32_t eig_sweeps;   /* block-Jacobi sweeps: first stage + 100 * refinement */
} gxy_step_info;

typedef struct gxy_ctx gxy_ctx;

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
gxy_status gxy_create(gxy_ctx **out, int device, void *hip_stream);
gxy_status gxy_destroy(gxy_ctx *ctx);

/* Device bytes needed to run the n points (largest single run). */
gxy_status gxy_workspace_bytes(gxy_ctx *ctx, const gxy_point *pts, int32_t n,
                               size_t *bytes);
/* Use caller-owned device memory (e.g. a torch tensor) as workspace. The
 * library never frees it; the caller keeps it alive while the context uses it.
 * Passing NULL returns to library-owned memory. */
gxy_status gxy_set_workspace(gxy_ctx *ctx, void *dev_ptr, size_t bytes);

/* Character coefficients t_n, n = -nmax..nmax (Ch. 3, eq. a_n as the
 * Fourier integral of the bond weight), computed on the device by the
 * nquad-point trapezoid rule; t is a host array of 2 nmax + 1 doubles. This
 * entry point takes the thesis's q = 2; runs with another harmonic compute
 * theirs from gxy_point.q (gxy_initial_tensor shows the resulting tensor). */
gxy_status gxy_char_coeffs(gxy_ctx *ctx, double beta, double delta,
                           int32_t nmax, int32_t nquad, double *t);

/* Initial site tensor T[l][r][u][d] (Ch. 3, final site-tensor equation) or an
 * impurity tensor (which = 0 pure, GXY_IMP_COS1, GXY_IMP_COS2; the two
 * impure-tensor equations of Ch. 3), built on the device and copied to the
 * host array out of (2 nmax + 1)^4 doubles. Unnormalised. */
gxy_status gxy_initial_tensor(gxy_ctx *ctx, const gxy_point *pt, int32_t which,
                              double *out);

/* One synchronous HOTRG run. */
gxy_status gxy_run(gxy_ctx *ctx, const gxy_point *pt, gxy_result *out);

/* n independent runs (points of a (beta, Delta, h, h1) scan, any mix of
 * Dcut, fields and precisions). With W > 1 workers (gxy_set_batch_workers,
 * else the GXY_BATCH_WORKERS environment variable, else 4) the runs are
 * taken longest first (cost ~ Dcut^7 x steps x placements) from a shared
 * queue by W host threads, each driving its own worker context: own
 * non-blocking stream, own device workspace (library-allocated, projection
 * chunks of at most 4 GiB), the caller's autotuned tiles. Small-Dcut runs
 * overlap the launch and host latency of the large ones. Workers keep to
 * their one stream; HIP maps streams onto GPU_MAX_HW_QUEUES hardware queues
 * per process (4 unless set before HIP starts), and streams that share a
 * queue run their kernels one after another, so W workers want at least W
 * queues. Results are in
 * input order and identical, bit for bit, to gxy_run of each point. Per-run
 * status in out[i].status (failed runs: NaN outputs); GXY_EPARTIAL if any
 * run failed, GXY_EDEVICE (remaining runs not started) on a device error. */
gxy_status gxy_run_batch(gxy_ctx *ctx, const gxy_point *pts, int32_t n,
                         gxy_result *out);

/* Size of the device scratch array behind gxy_run_noalloc (bytes). */
#define GXY_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* gxy_run for callers that cannot allocate device memory (code under HIP
 * graph capture of the surrounding work, tight serving loops, harnesses
 * that forbid hipMalloc): the same run and the same results as gxy_run,
 * with every device buffer carved from one file-scope scratch array of
 * GXY_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs
 * on until the process ends. The call makes no HIP allocation (no hipMalloc,
 * hipFree, pinned host memory, stream or event creation) and no torch
 * allocation; its host-side planning uses the C++ heap. Work runs on the
 * context's stream only (no side streams, one workgroup per eigensolver
 * sector) and the call returns when the run is done.
 * Limits and errors: a run whose workspace does not fit the array, even with
 * the projection split into the smallest chunks, returns GXY_EINVAL before
 * any device work (the last error names both sizes); other statuses as for
 * gxy_run. The array keeps the last call's contents; every buffer a run reads
 * is written by that run first. All calls on one device share that device's
 * array: calls that overlap in time on one device (two host threads, or two
 * contexts) race and must not be issued. The context's own workspace
 * (gxy_set_workspace or library-owned) is neither used nor changed. */
gxy_status gxy_run_noalloc(gxy_ctx *ctx, const gxy_point *pt, gxy_result *out);

/* Number of worker contexts gxy_run_batch uses (0 = default, at most 64). */
gxy_status gxy_set_batch_workers(gxy_ctx *ctx, int32_t workers);

/* Measure, for each Dcut in dcuts[0..n), the projection contractions with
 * 64 x 64, 128 x 128 and 256 x 128 output tiles (tile 64, 128, 256) on the
 * run templ (with that Dcut; its second run is timed, the first warms up)
 * and keep the fastest tile for later runs at that Dcut on this context
 * (and its batch workers). tiles[i] (optional) receives the choice,
 * ms[3 i .. 3 i + 2] (optional) the summed time of the D^7 products for 64,
 * 128 and 256. The tile does not change any result: every output element
 * is accumulated over the same k-slices in the same order. */
gxy_status gxy_autotune(gxy_ctx *ctx, const gxy_point *templ, const int32_t *dcuts,
                        int32_t n, int32_t *tiles, double *ms);

/* Per-step diagnostics of run `run` of the last gxy_run (run = 0) or
 * gxy_run_batch; writes min(cap, steps) entries and the count to *count. */
gxy_status gxy_step_log(gxy_ctx *ctx, int32_t run, gxy_step_info *out,
                        int32_t cap, int32_t *count);

/* Observables of Ch. 3 (eqs. spech, susc, mag) from the seven runs of one
 * (beta, Delta) point: lnz[3] = ln Z/V at beta-db, beta, beta+db;
 * m_h[2] = <cos theta> at h = hc-dh, hc+dh; m_h1[2] = <cos 2 theta> at
 * h1 = hc-dh1, hc+dh1. out[4] = (f, C_v, chi, chi_n). Evaluated on the device. */
gxy_status gxy_observables(gxy_ctx *ctx, int32_t npts, const double *beta,
                           const double *lnz, const double *m_h,
                           const double *m_h1, double dbeta, double dh,
                           double dh1, double *out);

const char *gxy_status_string(gxy_status s);
const char *gxy_last_error(gxy_ctx *ctx);

/* Last run's device timing of each phase, in milliseconds: [0] coefficients
 * and initial tensors, [1] environments, [2] eigensolver, [3] selection and
 * projector, [4] projection contractions, [5] norms/permutes/trace. Valid when
 * the environment variable GXY_TIMING is set during the run. */
gxy_status gxy_phase_times(gxy_ctx *ctx, double *ms6);

/* Accumulated device timing of the dominant contraction (the D^7 product
 * Y = X T of the projection, Ch. 2 eq. renormalizedT) over the runs issued
 * while GXY_TIMING or GXY_HOT_EVENTS was set: out4 = (launches, total milliseconds measured with
 * HIP events on the context's stream, algorithmic flops, algorithmic bytes).
 * reset != 0 clears the totals after reading. */
gxy_status gxy_hot_kernel_stats(gxy_ctx *ctx, double *out4, int32_t reset);

/* ------------------------------------------------------------------------
 * Learned surrogate of the phase diagram (not in the thesis, which motivates
 * cheaper scans of the (beta, Delta) plane in Ch. 3): a 2 -> 128 -> 128 -> 4
 * multilayer perceptron, SiLU after both hidden layers, linear output,
 * 17 412 FP32 parameters laid out W1[128][2], b1[128], W2[128][128], b2[128],
 * W3[4][128], b3[4] (row-major, layer maps a -> W a + b). Inputs
 * (beta, Delta); targets (f, C_v, chi, chi_n), the observables of Ch. 3
 * (eqs. spech, susc). Training is full-batch Adam on the mean squared error
 * of standardised targets, in FP32 on the device, reproducible bit for bit.
 * A surrogate belongs to the context it was created on and uses its device;
 * calls are ordered after the context stream's work and return when done.
 * ---------------------------------------------------------------------- */
typedef struct gxy_mlp gxy_mlp;

typedef struct {
  int32_t epochs;          /* Adam updates (full batch), >= 0                */
  float lr, beta1, beta2, eps; /* Adam step size and moment constants       */
  uint32_t log_targets;    /* bit c set: target column c enters as ln(y_c)   */
  int32_t standardize;     /* 1: inputs and (transformed) targets are
                              standardised with the training set's mean and
                              population standard deviation; 0: used as is  */
} gxy_train_cfg;

typedef struct {
  int32_t nbeta, ndelta;   /* candidate lattice, nbeta >= 3, ndelta >= 2     */
  double beta_lo, beta_hi; /* beta_i = lo + i (hi - lo) / (nbeta - 1)       */
  double delta_lo, delta_hi; /* likewise Delta_j                             */
  uint64_t seed;           /* SplitMix64 stream of the jitter               */
  double jitter;           /* 0..1: proposals move by jitter (2u - 1) / 2
                              lattice spacings along beta                   */
  int32_t cv_col, chi_col; /* target columns whose maxima are proposed      */
} gxy_propose_cfg;

/* New surrogate with Xavier-uniform weights drawn from the SplitMix64 stream
 * seeded with seed (weights of W1, W2, W3 in order; u = (z >> 11) 2^-53,
 * w = (2u - 1) sqrt(6 / (fan_in + fan_out))) and zero biases. */
gxy_status gxy_mlp_create(gxy_ctx *ctx, uint64_t seed, gxy_mlp **out);
gxy_status gxy_mlp_destroy(gxy_mlp *mlp);
/* Copy the 17 412 parameters out (get) and/or in (set); either may be NULL. */
gxy_status gxy_mlp_params(gxy_mlp *mlp, float *get, const float *set);
/* Train from the current parameters with a fresh Adam state. x: n x 2
 * (beta, Delta), y: n x 4 targets in physical units (row-major FP64);
 * columns selected by log_targets must be > 0. loss_hist (optional,
 * epochs floats): loss at the parameters before each update. The scaling
 * found here is kept for gxy_mlp_predict / gxy_mlp_propose. */
gxy_status gxy_mlp_train(gxy_mlp *mlp, const double *x, const double *y, int32_t n,
                         const gxy_train_cfg *cfg, float *loss_hist);
/* Loss and its gradient (17 412 floats, parameter layout) at the current
 * parameters for data already in network units (x: n x 2, y: n x 4, FP32). */
gxy_status gxy_mlp_grad(gxy_mlp *mlp, const float *x, const float *y, int32_t n,
                        float *grad, float *loss);
/* Predictions in physical units (n x 4, FP64) for raw (beta, Delta) rows;
 * bf16 = 1 runs the 128 x 128 layer on BF16 matrix cores, 0 all-FP32. */
gxy_status gxy_mlp_predict(gxy_mlp *mlp, const double *x, int32_t n, int32_t bf16,
                           double *y);
/* Scaling in use: out12 = x mean[2], y mean[4], x std[2], y std[4] (targets
 * after the log transform); *log_mask = the transformed columns. */
gxy_status gxy_mlp_scaling(gxy_mlp *mlp, double *out12, uint32_t *log_mask);
/* Two refinement points per Delta_j of the lattice: at the predicted maxima
 * along beta of columns cv_col and chi_col (BF16 inference). beta_delta
 * receives 2 ndelta rows (beta, Delta): row 2j the cv_col maximum, row 2j+1
 * the chi_col maximum. The first maximum wins ties; the vertex of the
 * parabola through it and its two neighbours moves it by at most half a
 * spacing; then the jitter is added and beta is clamped to the lattice. */
gxy_status gxy_mlp_propose(gxy_mlp *mlp, const gxy_propose_cfg *cfg, double *beta_delta);

#ifdef __cplusplus
}
#endif

#endif /* GXY_HOTRG_H */
