/*
 * ep.h -- C ABI of the MI355X expectation-propagation library for
 * three-dimensional Gaussian-process extinction mapping.
 *
 * Method: Sale & Magorrian, "Large-scale three-dimensional Gaussian process
 * extinction mapping" (arXiv:1708.09705).
 *
 * Model.  The unknown is the log extinction pseudo-density
 * f(x) = ln(rho kappa)(x) (Sec. 5: dA/ds = rho kappa) on a regular n^3 grid.
 * Its prior is a Gaussian process (Sec. 2) with a turbulence-shaped
 * covariance (Sec. 1: Kolmogorov spectrum truncated at the outer scale, here
 * a Matern nu = 1/3 kernel with length scale equal to the outer scale)
 * tapered to a compact support and made sparse by a Vecchia
 * (inverse-Cholesky) precision Q0.  Each star n at a known distance
 * (Sec. 4.1, simplified case) has extinction A_n = integral of exp(f) along
 * its sightline; its likelihood is N(A_obs_n | A_n, sigma_n^2).
 *
 * Inference is parallel expectation propagation (Sec. 4.1; App. A.2): one
 * Gaussian site per star in a_n = ln A_n, cavity -> tilted -> moment
 * matching, every site updated from the same posterior in a sweep.  The
 * posterior precision Q = Q0 + sum_n tau_n g_n g_n^T is factored by a
 * multifrontal Cholesky on the GPU; the posterior mean comes from the
 * triangular solves and the marginal variances (Sec. 5: maps of marginal
 * posterior mean and variance) from selected inversion.
 *
 * Conventions
 *  - Every call returns an ep_status (0 = success).  On failure
 *    ep_last_error(ctx) (or ep_last_error(NULL) for failures without a
 *    context) holds a message.
 *  - Host pointers, or device pointers on cfg.device for ep_init and every
 *    call on a context when cfg.pointers_on_device = 1.  The library copies
 *    every input it keeps; the caller owns every buffer it passes.
 *  - Grid node p = i + n (j + n k) sits at h (i, j, k), h = box/(n-1).
 *  - Work runs on the context's HIP stream; calls return after completion.
 *    A context is not thread-safe; distinct contexts are independent.
 */
#ifndef EP_H
#define EP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EP_OK = 0,
    EP_ERR_INVALID_ARG = -1, /* bad argument or configuration */
    EP_ERR_OOM = -2,         /* device allocation failed or exceeded hbm_cap_bytes */
    EP_ERR_NOT_PD = -3,      /* a pivot of the posterior precision was not positive */
    EP_ERR_DEVICE = -4,      /* HIP runtime error */
    EP_ERR_STATE = -5,       /* call not valid in the context's state */
    EP_ERR_NUMERIC = -6      /* non-finite value in the sites or the posterior */
} ep_status;

typedef enum { EP_LIK_EXTINCTION = 0, EP_LIK_GAUSS_LINEAR = 1, EP_LIK_GMM = 2 } ep_likelihood;
/* SELINV32: the factor, solves and sites in FP64 and the selected inversion's
 * dense block products (Sigma_21 = -Sigma_22 L21 L11^{-1}, Sigma_11) on FP32
 * MFMA with FP64 storage: operands rounded to FP32, products summed in FP32
 * over 64 terms at a time and those partial sums in FP64.  The marginal
 * variances and the cavities then carry FP32 rounding (about 1e-6 relative
 * on a 64^3 grid); the posterior mean does not. */
typedef enum { EP_PREC_FP64 = 0, EP_PREC_MIXED = 1, EP_PREC_SELINV32 = 2 } ep_precision;
typedef enum { EP_MOM_QUADRATURE = 0, EP_MOM_SURROGATE = 1 } ep_moments;
typedef enum { EP_MEAN_CONSTANT = 0, EP_MEAN_DISC_BUMP = 1 } ep_mean_fn;

typedef struct ep_config {
    /* grid */
    int32_t n;                 /* nodes per axis (>= 2) */
    double box_pc;             /* cube side L in pc; nodes span [0, L]^3 */
    double observer_pc[3];     /* observer position (the sightlines start here) */
    /* prior on f = ln(rho kappa) */
    double prior_mean;         /* constant mean m0, ln(mag/pc) */
    double prior_var;          /* variance sigma_f^2 */
    double outer_scale_pc;     /* Matern length scale (the outer scale) */
    double support_pc;         /* taper radius r_s: covariance is 0 beyond it */
    double vecchia_radius_pc;  /* conditioning radius rho; 0 means support_pc */
    /* forward model */
    double los_step_pc;        /* trapezoid steps are d/T <= this, T = ceil(d/step) */
    /* modes */
    int32_t likelihood;        /* ep_likelihood */
    int32_t precision;         /* ep_precision: FP64, or MIXED = FP32 factor on FP32 MFMA
                                  with FP64 diagonal pivots, FP64 refinement of the
                                  mean and FP64 selected inversion, or SELINV32 =
                                  FP64 factor with the selected inversion's block
                                  products on FP32 MFMA */
    int32_t moments;           /* ep_moments: QUADRATURE, or SURROGATE = gated network
                                  with quadrature fallback (needs ep_mlp_load) */
    /* EP controls */
    double damping;            /* delta in (0, 1]: site <- (1-delta) old + delta new */
    double cavity_var_floor;   /* cavity variance floor (Sec. 5), 0 = none */
    int32_t relinearize;       /* 1: relinearise each sweep at the posterior mean;
                                  0: freeze g_n, c_n at the prior mean */
    /* device */
    int32_t device;            /* HIP device ordinal */
    void *stream;              /* hipStream_t to run on; NULL = library-owned stream */
    int32_t leaf_size;         /* ordering: largest dissection leaf (0 = 512) */
    int64_t hbm_cap_bytes;     /* refuse to allocate more than this (0 = no cap) */
    int32_t profile_kernels;   /* 1: time every MFMA tile-kernel launch with HIP events */
    int32_t mixed_fp64_levels; /* mixed precision: factor the top k levels of the
                                  dissection tree in FP64 (0 = all levels FP32) */
    double surrogate_tol;      /* surrogate moments: accept a star when the network's
                                  moments and the Gauss-Hermite check agree to this */
    int32_t pointers_on_device; /* 0: the array arguments of ep_init and of every call
                                   on a context are host memory; 1: they are device
                                   memory on `device` (e.g. torch tensors), written and
                                   read before the call returns.  Arrays that need
                                   checks or host-side work (star inputs, sites, the
                                   linearisation point, z, point pairs, weights) are
                                   copied to the host first.  Context-free calls
                                   (ep_tilted_moments, ep_simulate, ep_mlp_*) always
                                   take host memory. */
    /* prior mean of f (Sec. 5): CONSTANT = prior_mean; DISC_BUMP = ln of an
     * exponential disc plus a Gaussian bump in rho kappa, whose five
     * parameters theta = (L, H, rho kappa_0, s_bump, A_bump) are inferred
     * with the field (EP over the field and phi = ln theta jointly, Sec. 4.1).
     * Geometry: the observer is in the disc mid-plane z = observer z at
     * Galactocentric radius sun_radius_pc and looks along +y away from the
     * Galactic centre; R = sqrt((R0 + y - y_o)^2 + (x - x_o)^2), h = z - z_o;
     * the bump is a slab across the line of sight at y - y_o = s_bump.
     *   rho kappa = rk0 exp(-(R - R0)/L - |h|/H) + A_b N(y - y_o; s_b, w^2) exp(-|h|/H).
     * DISC_BUMP needs precision FP64. */
    int32_t mean_fn;           /* ep_mean_fn */
    double theta_prior[5];     /* log-normal hyperprior means of theta (pc, pc, mag/pc, pc,
                                  mag); each hyperprior's sd equals its mean.  ep_simulate
                                  with DISC_BUMP draws around m(x; theta_prior). */
    double sun_radius_pc;      /* R0 (default 8000) */
    double bump_width_pc;      /* w, the bump's fixed standard deviation (default 400) */
    /* linearisation step r in (0, 1] (default 1): after a sweep the
     * linearisation point moves the fraction r of the way to the posterior
     * mean, fhat <- fhat + r (mu - fhat) (with DISC_BUMP the same step for
     * deltahat and phihat).  r = 1 puts it at the mean; r < 1 is a damped
     * Gauss-Newton step with the same fixed points, for fields whose full
     * steps settle into a 2-cycle.  Extinction and GMM likelihoods with
     * relinearize = 1 only. */
    double relin_step;
    /* 1: a sweep's results are bitwise reproducible run to run on the same
     * device and inputs.  The floating-point atomic adds of the sweep are
     * replaced by sums in a fixed order: the right-hand side node by node
     * over its stars; the forward solve's update rows node by node over the
     * level's fronts; the trailing updates are not split along K.  (The star
     * cliques are summed in a fixed order in either mode.)  Needs precision
     * FP64 and mean_fn CONSTANT; slower (the unsplit trailing updates).
     * 0: the default, atomic adds (results agree to rounding). */
    int32_t deterministic;
} ep_config;

/* Kinds of timed kernel launches (ep_sweep_stats.kernel_ms, with
 * profile_kernels = 1).  MFMA tile kernels: column-panel triangular solves,
 * in-panel rank updates, trailing updates after each panel, and the
 * task-list GEMM kernel (diagonal-block inverses and the selected-inversion
 * products).  Sparse kernels: zeroing of the fronts' lower tiles, the star
 * cliques' assembly into the fronts, extend-add of the update blocks, the
 * selected inversion's gather of the parent's Sigma, the cavity, and the
 * triangular-solve kernels. */
enum {
    EP_KK_TRSM = 0,
    EP_KK_INNER = 1,
    EP_KK_TRAIL = 2,
    EP_KK_GEMM = 3,
    EP_KK_MFMA = 4,            /* kinds below this one are the MFMA tile kernels */
    EP_KK_ZERO = 4,
    EP_KK_ASSEMBLE = 5,
    EP_KK_EXTEND = 6,
    EP_KK_GATHER = 7,
    EP_KK_CAVITY = 8,
    EP_KK_SOLVE = 9,
    EP_KK_COUNT = 10
};

typedef struct ep_sweep_stats {
    double ms_linearise;       /* line-of-sight linearisation */
    double ms_assemble;        /* Q and b assembly */
    double ms_factor;          /* multifrontal Cholesky + diagonal-block inverses */
    double ms_solve;           /* triangular solves -> posterior mean */
    double ms_selinv;          /* selected inversion -> Sigma on the front pattern */
    double ms_star;            /* per-star phase: cavity + tilted moments + site update */
    double ms_total;           /* the whole sweep */
    int64_t updated;           /* sites replaced */
    int64_t skipped_cavity;    /* cavity precision <= 0 */
    int64_t skipped_negsite;   /* new site precision < 0 or non-finite */
    double max_dtau;           /* max |change of site precision| */
    double max_dmu;            /* max |posterior mean - previous linearisation point| */
    double mfma_ms;            /* summed duration of the MFMA tile-kernel launches (profile_kernels) */
    int64_t mfma_launches;     /* number of those launches */
    int32_t refine_iters;      /* mixed precision: FP64 refinement rounds of the mean */
    double refine_residual;    /* mixed precision: final ||b - Q mu|| / ||b|| */
    int64_t surrogate_fallbacks; /* surrogate moments: stars sent to the quadrature */
    double kernel_ms[EP_KK_COUNT];        /* timed launches by kind (EP_KK_*) */
    int64_t kernel_launches[EP_KK_COUNT]; /* mfma_launches split by kind */
} ep_sweep_stats;

typedef struct ep_structure_stats {
    int64_t n_nodes;
    int64_t n_stars;
    int64_t nnz_g;             /* total sightline support size */
    int64_t n_fronts;
    int32_t n_levels;
    int64_t front_elems;       /* sum of m^2 over fronts (factor / Sigma storage) */
    int64_t max_front;         /* largest front order */
    double factor_flops;       /* partial Cholesky flops of all fronts */
    double selinv_flops;       /* selected-inversion flops, diagonal-block
                                  inverses included (the EP_KK_GEMM work) */
    double trail_flops;        /* trailing-update share of factor_flops
                                  (the EP_KK_TRAIL work) */
    int64_t device_bytes;      /* bytes the context holds on the device */
    int64_t front_elems_lower; /* elements of the fronts' lower-triangular 64 x 64 tiles */
    int64_t update_elems;      /* sum over fronts of nr (nr + 1) / 2: the update blocks' lower triangles */
    int64_t offdiag_elems;     /* sum over fronts of nr nv: the factor's off-diagonal blocks */
    int64_t x_elems;           /* sum over fronts of nvpad^2: the pivot blocks' inverses */
    int64_t clique_pairs;      /* sum over stars of |P|(|P| + 1) / 2: the cliques' lower triangles */
} ep_structure_stats;

typedef struct ep_ctx ep_ctx;

/* Fill *cfg with defaults: n=16, box 1000 pc, observer at the centre of the
 * y=0 face, m0=-7, variance 1, outer scale 100 pc, support 150 pc,
 * step 2 pc, extinction likelihood, FP64, quadrature, damping 1. */
void ep_config_default(ep_config *cfg);

/* Create a context: build the Vecchia prior, the sightline supports, the
 * nested-dissection ordering and the front layout (host), upload the
 * structure, and set every site to zero and the linearisation point to the
 * prior mean.  xyz: n_stars x 3 positions (pc, cube frame) at known
 * distances (Sec. 4.1); A_obs: observed extinction (mag; in the
 * gauss_linear mode the observed log-extinction); sigma: 1-sigma noise
 * (> 0).  With likelihood GMM (unknown distances) xyz are the catalogue
 * positions, A_obs and sigma are unused (may be NULL) and ep_set_gmm must
 * give the per-star mixtures before the first sweep.  Errors: INVALID_ARG
 * (bad config, non-finite input, star outside the cube or at the observer),
 * OOM, DEVICE.  n_stars = 0 is allowed: the posterior is then the prior. */
int ep_init(const ep_config *cfg, int64_t n_stars, const double *xyz, const double *A_obs,
            const double *sigma, ep_ctx **out);

/* One parallel EP sweep (App. A.2, parallel procedure): linearise every
 * sightline at the current point, assemble and factor the posterior
 * precision, posterior mean and selected inverse, then for every star the
 * cavity, the tilted moments (Sec. 4.1) and the damped site update; finally
 * move the linearisation point to the posterior mean.  stats may be NULL.
 * On NOT_PD or NUMERIC the sites and the linearisation point are left as
 * they were before the call. */
int ep_sweep(ep_ctx *ctx, ep_sweep_stats *stats);

/* Posterior mean of f at every node (n^3 doubles, node order) with the
 * current sites at the current linearisation point.  Changes no state. */
int ep_posterior_mean(ep_ctx *ctx, double *out);

/* Marginal posterior variance of f at every node (n^3 doubles). */
int ep_marginal_var(ep_ctx *ctx, double *out);

/* Release everything.  NULL is allowed. */
void ep_free(ep_ctx *ctx);

/* Posterior of the mean parameters (mean_fn DISC_BUMP), recomputed like
 * ep_posterior_mean: mean (5) and covariance (5 x 5 row-major, may be NULL)
 * of phi = ln theta, theta = (L, H, rho kappa_0, s_bump, A_bump).  The border
 * of the joint precision is eliminated by its Schur complement after the
 * grid factorization (five extra solves).  STATE with mean_fn CONSTANT;
 * NOT_PD if the Schur complement is not positive definite. */
int ep_theta(ep_ctx *ctx, double *mean, double *cov);

/* Message of the last failure on ctx (or of the calling thread when ctx is
 * NULL).  Never NULL. */
const char *ep_last_error(const ep_ctx *ctx);

/* Site natural parameters (tau_n, nu_n) per star: get copies them out, set
 * replaces them (checkpoint / resume). */
int ep_get_sites(ep_ctx *ctx, double *tau, double *nu);
int ep_set_sites(ep_ctx *ctx, const double *tau, const double *nu);

/* Unknown distances (Sec. 4.2 general case; likelihood GMM): per-star
 * Gaussian mixtures over (l, b) = (ln distance / pc, log-extinction to that
 * distance), K (1..8) components per star, comps n_stars x K x 6 rows
 * (w, m_l, m_b, C_ll, C_lb, C_bb): weights >= 0 with a positive sum, C_bb > 0,
 * C positive definite (or C_ll = C_lb = 0: the distance is known).  The
 * tilted distribution sums over the components and integrates over the
 * distance s.  The site stays on a_n = ln A to the catalogue position
 * (distance s~); the log-extinction at distance s is
 * a_n + ln A(s; fhat) - ln A(s~; fhat), from the sightline forward model at
 * the linearisation point extended past the star (the star's own steps to s~,
 * then steps of los_step_pc to the cube's face; the trapezoid sum to the last
 * sample below s plus the partial trapezoid to s); distances past the cube's
 * face carry no likelihood.  Per component the integral over a_n is closed
 * form and the one over l = ln s a composite 16-panel, 16-node
 * Gauss-Legendre rule over m_l +- 8 sd(l).  A star whose every component lies
 * outside the cube gets lnZ = -inf and keeps its site.  May be called again
 * (e.g. with another K).  Errors: INVALID_ARG (also when the extended
 * sightlines and K need more than the kernel's 64 KB of LDS), STATE
 * (likelihood not GMM), OOM, DEVICE. */
int ep_set_gmm(ep_ctx *ctx, int32_t K, const double *comps);

/* Linearisation point: fhat (n^3 doubles), followed with mean_fn DISC_BUMP
 * by phihat, the 5 log-parameters about which the mean is linearised. */
int ep_get_linpoint(ep_ctx *ctx, double *f);
int ep_set_linpoint(ep_ctx *ctx, const double *f);

/* Per-star quantities of the last sweep: ln A_n at the linearisation
 * point, cavity mean and variance of a_n, and the tilted moments
 * (ln Z, mean, variance).  Each array has n_stars doubles; any may be
 * NULL. */
int ep_star_state(ep_ctx *ctx, double *lnA, double *cav_mu, double *cav_var, double *lnZ,
                  double *tmean, double *tvar);

/* Batch tilted moments (the per-star moment matching of Sec. 4.1), without
 * a context.  mode: ep_likelihood.  Inputs and outputs: n doubles each,
 * host memory. */
int ep_tilted_moments(int32_t mode, int64_t n, const double *mu_c, const double *v_c,
                      const double *A, const double *sigma, double *lnZ, double *mean,
                      double *var, int32_t device);

/* Synthetic observations with the library's own arithmetic (for
 * benchmarks): f_true = m0 + (I-B)^{-1} D^{1/2} xi (exact draw from the
 * Vecchia prior; with mean_fn DISC_BUMP m0 is the field m(x; theta_prior)) and A_obs = A(f_true) + sigma * eps (extinction) or
 * c_n + g_n.f_true + sigma * eps with g, c at the prior mean
 * (gauss_linear).  xi: n^3 deviates; xyz, sigma, eps per star.  Outputs:
 * f_true (n^3) and A_obs (n_stars), either may be NULL. */
int ep_simulate(const ep_config *cfg, int64_t n_stars, const double *xyz, const double *sigma,
                const double *eps, const double *xi, double *f_true, double *A_obs);

/* ---- Tilted-moment surrogate (the per-star moment matching of Sec. 4.1) ----
 * A 4-128-128-128-3 SiLU network predicts corrections to a Gaussian baseline
 * of the tilted distribution (the likelihood linearised in a = ln A at
 * ln max(A, sigma), times the cavity).  Weights: EP_MLP_NPARAM floats, in
 * the order W1 (4x128) b1 W2 (128x128) b2 W3 b3 W4 (128x3) b4, then the
 * feature mean and std (4 + 4) and the target mean and std (3 + 3).
 * Inference runs with BF16 operands on MFMA.  The gate: a 20-node
 * Gauss-Hermite rule centred at the prediction computes the moments of the
 * true integrand, a 32-node rule re-centred at those moments checks them, and
 * the star is accepted when the passes agree to surrogate_tol (relative in
 * var and in mean on the scale max(|mean|, sd), absolute in ln Z) with an
 * analytic bound on the tails beyond 8 sd added, and the predicted variance
 * is within a factor 4; accepted stars take the second
 * pass's moments, the others fall back to the quadrature. */
#define EP_MLP_NPARAM 34065

typedef struct ep_mlp_hyper {
    int32_t epochs;            /* passes over the data */
    int32_t batch;             /* samples per Adam step */
    double lr;                 /* peak learning rate (cosine decay to 0) */
    uint64_t seed;             /* initialisation and shuffling */
} ep_mlp_hyper;

/* Train on n tuples.  inputs: n x 4 (cavity mean mu_c, cavity variance v_c,
 * observed A, noise sigma); targets: n x 3 (ln Z, mean, variance of the
 * tilted distribution).  Mean squared error on the standardised baseline
 * corrections; Adam.  weights_out: EP_MLP_NPARAM floats; loss_per_epoch:
 * epochs doubles (may be NULL). */
int ep_mlp_train(const ep_mlp_hyper *hp, int64_t n, const double *inputs, const double *targets,
                 float *weights_out, double *loss_per_epoch, int32_t device);

/* Gated surrogate moments for n tuples (inputs as above).  out3: n x 3
 * (ln Z, mean, var), the Gauss-Hermite moments where accepted and the
 * network's otherwise; errest: the gate's error estimate; accepted: 1/0.
 * errest and accepted may be NULL.  weights == NULL centres the gate at the
 * analytic baseline instead of the network (what the network is measured
 * against). */
int ep_mlp_predict(const float *weights, int64_t n, const double *inputs, double tol, double *out3,
                   double *errest, int32_t *accepted, int32_t device);

/* One forward and backward pass on already standardised features (n x 4)
 * and targets (n x 3): the loss (mean over samples of the summed squared
 * error) and its gradient for the trainable prefix of the weights. */
int ep_mlp_loss_grad(const float *weights, int64_t n, const float *xstd, const float *ystd, double *loss,
                     float *grad, int32_t device);

/* ---- For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc) ----
 * ep_mlp_predict_noalloc: ep_mlp_predict on device memory with no device
 * allocation.  weights (EP_MLP_NPARAM floats, or NULL for the gate centred at
 * the analytic baseline), inputs (n x 4), out3 (n x 3), errest (n) and
 * accepted (n) are device buffers on `device`, owned by the caller; errest
 * and accepted may be NULL.  stream: the hipStream_t to run on (NULL = the
 * device's null stream); the call returns after completion.  Same results as
 * ep_mlp_predict on the same data.  The BF16 copy of the hidden layers, the
 * inputs split per field, the zero site arrays and an error counter live in
 * one static device array of about 40 MB that every GPU the library runs on
 * holds until the process ends; it is looked up on the first call on each
 * device.  Calls on one GPU share that array: calls that overlap on one GPU
 * (other host threads, other streams) race and must be serialised by the
 * caller.  Errors: INVALID_ARG (n < 0 or n > EP_NOALLOC_MAX_TUPLES, NULL
 * buffers, tol <= 0, device out of range, or a tuple with a non-finite mean or
 * observation or v_c <= 0 or sigma <= 0, checked on the device before the
 * network runs; outputs are then untouched), DEVICE. */
#define EP_NOALLOC_MAX_TUPLES 1048576
int ep_mlp_predict_noalloc(const float *weights, int64_t n, const double *inputs, double tol, double *out3,
                           double *errest, int32_t *accepted, int32_t device, void *stream);

/* Give a context the network used when cfg.moments = EP_MOM_SURROGATE. */
int ep_mlp_load(ep_ctx *ctx, const float *weights);

/* Structure and memory figures of a context. */
int ep_structure(const ep_ctx *ctx, ep_structure_stats *out);

/* Structure, work and memory of a configuration without a device: the
 * host analysis of ep_init (sightline supports, nested dissection, the
 * multifrontal layout of the posterior precision's factor) on the same
 * inputs, with the device memory ep_init would take counted instead of
 * allocated.  Host memory and time grow with the stars' supports and the
 * fronts' R lists (about 2 GB and a minute for 128^3 nodes and 10^6 stars).
 * Errors: INVALID_ARG (config or star positions), STATE (analysis). */
typedef struct ep_plan_stats {
    int64_t n_nodes, n_stars;
    int64_t nnz_g;             /* total sightline support size */
    int64_t max_support;       /* largest sightline support (ep_init refuses > 1300) */
    int64_t n_fronts;
    int32_t n_levels;
    int64_t max_front;         /* largest front order (padded) */
    int64_t max_separator;     /* largest set of pivots of one front */
    int64_t front_elems;       /* sum of m^2: the fronts as stored (full squares) */
    int64_t front_elems_lower; /* the fronts' lower-triangular 64 x 64 tiles only */
    int64_t nnz_L;             /* nonzeros of the Cholesky factor: sum nv(nv+1)/2 + nv nr */
    int64_t x_elems;           /* inverses of the pivot blocks (sum nvpad^2) */
    int64_t w_elems;           /* selected-inversion scratch (largest level) */
    double factor_flops;       /* partial Cholesky flops of all fronts */
    double selinv_flops;       /* selected-inversion flops, diagonal-block inverses included */
    double trail_flops;        /* trailing-update share of factor_flops */
    int64_t device_bytes;      /* device memory of an FP64 context (without its GEMM task lists) */
    int64_t device_bytes_mixed;/* the same with the FP32 copy of the fronts (precision MIXED) */
} ep_plan_stats;
int ep_plan(const ep_config *cfg, int64_t n_stars, const double *xyz, ep_plan_stats *out);

/* ---- Map prediction from the posterior (Sec. 5: maps of extinction and
 * of the pseudo-density rho kappa = e^f) ----
 * Each call, like ep_posterior_mean, recomputes q(f) = N(mu, Sigma) from the
 * current sites at the current linearisation point and changes no state.
 * Outputs are arrays owned by the caller (host, or device memory with
 * pointers_on_device), in node order. */

/* The elimination order: perm[i] is the grid node eliminated i-th (N int32). */
int ep_ordering(const ep_ctx *ctx, int32_t *perm);

/* Posterior moments of rho kappa = e^f at every node (lognormal under q):
 * mean = exp(mu + v/2), var = (e^v - 1) exp(2 mu + v). */
int ep_density_moments(ep_ctx *ctx, double *mean, double *var);

/* Extinction A(x) from the observer to every grid node x, by the sightline
 * forward model (trapezoid at los_step_pc, trilinear field; 0 at the
 * observer's own node).  mean: the exact posterior mean (each sample point
 * s contributes its weight times exp(m(s) + v(s)/2), m and v from mu and
 * the Sigma block of the point's cell).  var (may be NULL): the sample
 * variance (divisor n_samples - 1) of A over posterior draws
 * f = mu + L^{-T} z_k, k < n_samples (>= 2), where z (n_samples x N
 * standard normals, caller-drawn) is consumed in elimination order
 * (ep_ordering); in mixed precision the draws use the FP32 factor.
 * The factor's pattern holds every cell's corners pairwise (ep_init adds
 * them), so Sigma is there for every sample point.
 * Errors: INVALID_ARG (n_samples < 2 with var, non-finite z), NOT_PD, OOM,
 * DEVICE; STATE only if a cell's Sigma block came out non-finite. */
int ep_extinction_map(ep_ctx *ctx, int32_t n_samples, const double *z, double *mean, double *var);

/* Joint predictive of the pseudo-density at n_pairs pairs of points
 * (x, x'), e.g. 10 pc apart (Sec. 5 density maps): xyz2 is n_pairs x 6
 * (x then x', pc, inside the cube); out5 is n_pairs x 5: E[rho(x)],
 * E[rho(x')], Var[rho(x)], Var[rho(x')], Cov[rho(x), rho(x')] of the
 * lognormal pair, from the trilinear field's Gaussian moments.  The two
 * points' cells (cell index clamp(floor(s/h), 0, n-2) per axis) must be the
 * same or touch (indices at most 1 apart per axis), which holds for points
 * up to one grid spacing apart; the factor's pattern then holds Sigma among
 * all 16 corners.  Errors: INVALID_ARG (a point outside the cube or
 * non-finite, cells that do not touch), NOT_PD, OOM, DEVICE; STATE only if
 * a Sigma entry came out non-finite. */
int ep_point_predict(ep_ctx *ctx, int64_t n_pairs, const double *xyz2, double *out5);

/* ---- The paper's sparse approximation: PITC sub-catalogue EP with a PIC
 * predictive (Sec. 4.1, App. A.1, App. B, App. C) ----
 * Needs a context with likelihood GAUSS_LINEAR: the observed
 * log-extinctions a~_n ~ N(a_n, sigma_n^2) with a_n = c_n + g_n . f the
 * sightline linearised at the prior mean (Sec. 4.1's Gaussian case), or
 * EXTINCTION with mean_fn CONSTANT (below),
 * f ~ N(m, K), K the tapered covariance between nodes (not the Vecchia
 * precision: this path is the paper's alternative to it).  Stars are split
 * into sub-catalogues k; u = f at R inducing nodes.  Blocks are independent
 * given u (PITC); EP keeps one Gaussian site per sub-catalogue, the site of
 * p(u | a~_k) / p(u) (the conditional with the minus sign the Gaussian
 * conditional needs; App. B prints a plus).  With mean_fn CONSTANT, m = m0
 * and the sites are on u; with mean_fn DISC_BUMP the prior mean is the
 * disc + bump function linearised at the hyperprior mean, m = mhat + J psi,
 * and the sites are on (u, psi) (the paper's q(u, Theta)), psi = ln theta -
 * phihat with its log-normal hyperprior.  Every block's tilted distribution
 * is Gaussian, so one undamped sweep reaches the fixed point.
 * With the extinction likelihood, A_n ~ N(e^{a_n}, sigma_n^2), every star
 * keeps its own Gaussian site on a_n (the context's star sites, as on the
 * grid path; ep_sites / ep_set_sites read and write them) and the
 * sub-catalogues enter through the PITC prior of a: a pass builds q(u) and
 * each star's posterior marginal of a_n from the current sites, then updates
 * every site from its cavity and tilted moments (damped by 'damping'; the
 * grid path's skip rules and cavity_var_floor).  Several passes are needed;
 * lnZ is NaN; ep_pitc_inducing and ep_pitc_predict rebuild q(u) from the
 * current sites.  (The paper keeps one site per sub-catalogue and samples
 * its tilted distribution.)
 * Memory: per sub-catalogue O((N_k + R + P_k) N_k + V_k (V_k + R + P_k))
 * doubles, V_k the nodes its sightlines touch and P_k the nodes it predicts
 * (with the extinction likelihood N_k more rows of N_k).
 *
 * ep_pitc_setup: star_block (n_stars int32, values 0..n_blocks-1, every
 * block non-empty), inducing (n_inducing >= 1 distinct node ids),
 * node_block (n^3 int32: the sub-catalogue whose stars each node's
 * prediction conditions on).  Plans and allocates; replaces an earlier set-up
 * and its sites.  Errors: INVALID_ARG (ranges, empty block, duplicate
 * inducing node, likelihood GMM, EXTINCTION with DISC_BUMP), OOM/DEVICE.
 * With the mean parameters the pass takes the context's mean linearised at
 * the hyperprior mean; once grid sweeps (ep_sweep) have moved that
 * linearisation (the Gaussian mode re-linearises the mean unless relinearize
 * = 0), ep_pitc_setup and the calls below return STATE.
 * ep_pitc_sweep: one parallel pass over the sub-catalogues from the same
 * q(u); sites damped by 'damping' in (0, 1] in natural parameters (the first
 * sweep starts from zero sites).  lnZ (may be NULL): the PITC log marginal
 * likelihood ln p(a~) = ln int p(u) prod_k p(a~_k | u) du.  Errors: STATE (no
 * set-up), INVALID_ARG (damping), NOT_PD (a block or K_uu not positive
 * definite), DEVICE.
 * ep_pitc_inducing: mean (R) and covariance (R x R, row-major) of q(u), in
 * the order of 'inducing'.  ep_pitc_predict: PIC predictive mean and
 * variance of f at every node (N each), f_p | a~_i, u from the joint
 * Gaussian of (f_p, a~_i, u) for i = node_block[p], integrated over q(u).
 * Both: STATE before the first sweep.  Arrays are caller-owned, host or
 * device per pointers_on_device. */
typedef struct ep_pitc_stats {
    int64_t n_blocks, n_inducing;
    int64_t max_block_stars;   /* largest N_k */
    int64_t max_block_nodes;   /* largest V_k */
    double sweep_flops;        /* algorithmic flops of one ep_pitc_sweep (unpadded sizes) */
    double predict_flops;      /* of one ep_pitc_predict */
    int64_t device_bytes;      /* the block pass's device memory */
} ep_pitc_stats;

int ep_pitc_setup(ep_ctx *ctx, int32_t n_blocks, const int32_t *star_block, int64_t n_inducing,
                  const int32_t *inducing, const int32_t *node_block);
int ep_pitc_sweep(ep_ctx *ctx, double damping, double *lnZ);
int ep_pitc_inducing(ep_ctx *ctx, double *mean, double *cov);
int ep_pitc_predict(ep_ctx *ctx, double *mean, double *var);
/* Mean (5) and covariance (5 x 5, row-major) of phi = ln theta under
 * q(u, Theta) (mean_fn DISC_BUMP).  STATE before the first sweep or with a
 * constant mean. */
int ep_pitc_theta(ep_ctx *ctx, double *mean, double *cov);
/* Sizes and algorithmic flop counts of the current set-up (STATE without one). */
int ep_pitc_info(const ep_ctx *ctx, ep_pitc_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* EP_H */
