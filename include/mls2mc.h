/*
 * mls2mc.h - C ABI of the MI355X (gfx950) library for the hot path of
 * Multilevel Sequential^2 Monte Carlo (Latz, Papaioannou, Ullmann,
 * "Multilevel Sequential^2 Monte Carlo for Bayesian Inverse Problems",
 * J. Comp. Phys.).
 *
 * The forward model is the one of the paper's Sec. 5: the log-permeability
 * theta(x) is a truncated Karhunen-Loeve expansion with N(0,1) coefficients,
 * kappa = exp(theta), and -div(kappa grad p) = f on (0,1)^2 with p = 0 on the
 * boundary and f = 1, discretised by P1 elements on the uniform mesh with
 * 2 n^2 triangles, n = 2^l; the observations are point values of p.  The
 * sampler pieces are those of Secs. 2-4: the Gaussian potential, the
 * ESS-adaptive tempering / bridging step, resampling and the Markov move
 * (here pCN).
 *
 * Conventions for every call:
 *  - Return value: MLS2MC_OK (0) or a positive status code below.  On error
 *    mls2mc_last_error() returns a message (thread-local, valid until the
 *    next call on the same thread).  No C++ exception crosses the ABI.
 *  - Array arguments are DEVICE pointers (memory of the context's GPU, e.g.
 *    from hipMalloc or a torch CUDA tensor) unless marked "host".  They are
 *    owned by the caller, contiguous, row-major and particle-major, and must
 *    stay valid until the work on `stream` has completed.  The library never
 *    frees caller memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work on it and return without waiting, except where stated.  Device
 *    scratch owned by the context is reused across calls, so calls on one
 *    context must not run concurrently on different streams.
 *  - Random numbers are inputs (normals, uniforms), except in mls2mc_run,
 *    which draws them with Philox4x32-10 keyed by the seed.
 *
 * Element ordering on level l (n = 2^l): cell (i,j), 0 <= i,j < n, is cut by
 * the diagonal from node (i,j) to (i+1,j+1); element 2(j n + i) is the lower
 * triangle {(i,j),(i+1,j),(i+1,j+1)}, element 2(j n + i)+1 the upper
 * triangle {(i,j),(i+1,j+1),(i,j+1)}; n_e(l) = 2 n^2.  Interior unknowns
 * (i,j), 1 <= i,j <= n-1, are ordered (j-1)(n-1)+(i-1); M(l) = (n-1)^2.
 * Observation o = (b-1) m + (a-1) is the point (a/(m+1), b/(m+1)).
 */
#ifndef MLS2MC_H
#define MLS2MC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define MLS2MC_OK 0
#define MLS2MC_EINVAL 1    /* bad shape, pointer, level or value           */
#define MLS2MC_ENOMEM 2    /* device or host allocation failed             */
#define MLS2MC_EDEVICE 3   /* a HIP runtime call failed                    */
#define MLS2MC_ENOTCONV 4  /* a solve did not converge or was non-finite   */
#define MLS2MC_ESINGULAR 5 /* all weights vanished / ESS collapse          */

/* ---- precision forms ---- */
#define MLS2MC_FP64 0  /* FP64 KL GEMM (MFMA), FP64 multigrid-PCG        */
#define MLS2MC_MIXED 1 /* BF16 KL GEMM (MFMA, FP32 accumulation), FP32
                          stencil/smoothing/inner PCG, FP64 residual and
                          iterative refinement, FP64 coarsest solve       */

/* ---- prior covariances (Sec. 5) ---- */
#define MLS2MC_COV_SEPEXP 0   /* sigma2 exp(-|dx1|/c) exp(-|dx2|/c): KL modes in
                                 closed form (roots of the 1-D eigen-equation) */
#define MLS2MC_COV_MATERN32 1 /* Matern, smoothness 3/2, the prior of the
                                 paper's elliptic examples (Sec. 5):
                                 sigma2 (1 + sqrt(6) r/lam) exp(-sqrt(6) r/lam),
                                 r = |x - x'|.  KL modes by the Nystrom method
                                 on the kl_quad x kl_quad midpoint grid; the
                                 eigenvectors are taken parity definite under
                                 x1 -> 1-x1 and x2 -> 1-x2 (paired eigenvalues:
                                 the one odd in x1 first), with the sign that
                                 makes sum_q g_q v_q > 0 for
                                 g_q = frac((q+1)^2 0.6180339887498949) - 1/2,
                                 q = b m + a over the grid points
                                 ((a+1/2)/m, (b+1/2)/m).  The basis at the
                                 element centroids is the Nystrom extension
                                 of each eigenvector.                         */

/* ---- boundary-value problems (Sec. 5) ---- */
#define MLS2MC_BC_DIRICHLET 0 /* -div(kappa grad p) = 1, p = 0 on the whole
                                 boundary; unknowns (i, j), 1 <= i, j <= n-1  */
#define MLS2MC_BC_FLOW_CELL 1 /* -div(kappa grad p) = 0, p = 0 at x1 = 0,
                                 p = 1 at x1 = 1, no flow through x2 = 0 and
                                 x2 = 1 (Example 5.3).  Unknowns (i, j),
                                 1 <= i <= n-1, 0 <= j <= n, ordered
                                 u = j (n-1) + (i-1).  kappa -> c kappa leaves
                                 p unchanged, so a constant prior mean of
                                 log kappa drops out                          */

/* ---- kinds of mls2mc_kl_field output ---- */
#define MLS2MC_FIELD_LOG_F64 0   /* a = theta B (double)                   */
#define MLS2MC_FIELD_KAPPA_F64 1 /* kappa = exp(a) (double)                */
#define MLS2MC_FIELD_KAPPA_F32 2 /* kappa = exp(a), BF16 GEMM (float)      */

typedef struct mls2mc_ctx mls2mc_ctx;

typedef struct {
    int l_min, l_max;  /* levels used, 1 <= l_min <= l_max <= 10 (h = 2^-l)  */
    int K;             /* KL terms, 1 <= K <= 512                            */
    double sigma2;     /* prior field variance (> 0)                         */
    double corr_len;   /* correlation length: c of the separable exponential
                          covariance sigma2 exp(-|dx1|/c) exp(-|dx2|/c), or
                          lam of the Matern covariance (see cov)             */
    int m;             /* observation grid side, N_obs = m*m, 1 <= m <= 32   */
    double sigma_n;    /* noise standard deviation, Gamma = sigma_n^2 I (> 0)*/
    int precision;     /* MLS2MC_FP64 or MLS2MC_MIXED                        */
    double rtol;       /* relative solver tolerance on the preconditioned
                          residual norm sqrt((r, V r) / (r0, V r0)), V the
                          multigrid cycle; 0 selects 1e-11 (FP64) / 1e-10
                          (MIXED, measured on the FP64 residual of the
                          iterative refinement)                             */
    int max_iters;     /* PCG iteration cap; 0 selects 200                   */
    int cov;           /* prior covariance: MLS2MC_COV_SEPEXP (0) or
                          MLS2MC_COV_MATERN32                                */
    int kl_quad;       /* MLS2MC_COV_MATERN32: side m of the Nystrom midpoint
                          grid (even, 4..128, K <= m*m); 0 selects 64.  Must
                          be 0 for MLS2MC_COV_SEPEXP                         */
    int bc;            /* boundary-value problem: MLS2MC_BC_DIRICHLET (0) or
                          MLS2MC_BC_FLOW_CELL (FP64 only; not with the
                          batched entry points)                              */
} mls2mc_problem;

/* Create a context on the current HIP device: builds the KL modes (roots of
 * the 1-D eigen-equation, or the Nystrom eigenpairs of the Matern operator;
 * Sec. 5 truncated KL expansion), the basis tables
 * B_l[k, e] = sqrt(lambda_k) phi_k(centroid_e) for l_min..l_max on the GPU,
 * and the observation tables.  *out receives the context.  Synchronous.    */
int mls2mc_create(const mls2mc_problem* p, mls2mc_ctx** out);
/* Free the context and all its device memory.  Synchronous.  NULL is OK.   */
int mls2mc_destroy(mls2mc_ctx* ctx);
const char* mls2mc_last_error(void);
/* library version string, e.g. "mls2mc 1.0 gfx950"                         */
const char* mls2mc_version(void);

/* KL eigenvalues lambda_k (descending, host array of K doubles), e.g. for
 * the paper's relative error with Lambda^{1/2} weights (Sec. 5.1).        */
int mls2mc_kl_eigenvalues(const mls2mc_ctx* ctx, double* lambda_out);

/* Observation count and level sizes (host queries).                        */
int mls2mc_n_obs(const mls2mc_ctx* ctx);
int64_t mls2mc_n_elem(int l);     /* 2 * 4^l                              */
int64_t mls2mc_n_unknowns(int l); /* (2^l - 1)^2                          */
/* unknowns of level l under the context's boundary-value problem:
 * (2^l - 1)^2, or (2^l - 1)(2^l + 1) for the flow cell; -1 on bad input   */
int64_t mls2mc_ctx_n_unknowns(const mls2mc_ctx* ctx, int l);

/* KL field (Sec. 5, truncated KL expansion; Sec. 2.2 discretisation):
 * out[q, e] = sum_k theta[q, k] B_l[k, e] for q < N, e < n_e(l), evaluated
 * at the element centroids, as a GEMM on the matrix cores.  theta: N x K
 * double.  kind selects the output: the log-field (double), kappa = exp(a)
 * (double), or kappa from the BF16 GEMM with FP32 accumulation (float).
 * Returns EINVAL for l outside [l_min, l_max], N < 0 or NULL pointers with
 * N > 0.                                                                   */
int mls2mc_kl_field(mls2mc_ctx* ctx, int l, int64_t N, const double* theta, void* out,
                    int kind, void* stream);

/* Forward response G_l(theta) = O(p) (Sec. 2.1 forward response operator;
 * Sec. 5 model): KL field, kappa = exp(a), solve A_l(kappa) p = b with
 * multigrid-preconditioned CG, observe p at the N_obs points.  The
 * boundary-value problem is the context's (bc): the Dirichlet problem with
 * f = 1, or the flow cell (Example 5.3), whose observations see p = 0 and
 * p = 1 on its Dirichlet edges.
 * theta: N x K double; G_out: N x N_obs double.
 * status_out (N int8, may be NULL): 0 converged, 1 not converged within
 * max_iters, 2 non-finite.  iters_out (N int32, may be NULL): PCG
 * iterations (MIXED: inner iterations summed over refinement sweeps).
 * Returns EINVAL on bad arguments; non-convergence is reported only through
 * status_out (the call itself returns OK).                                 */
int mls2mc_forward(mls2mc_ctx* ctx, int l, int64_t N, const double* theta, double* G_out,
                   int8_t* status_out, int32_t* iters_out, void* stream);

/* Forward response from a given coefficient batch (skips the KL field):
 * kappa: N x n_e(l) double, one positive value per element; G_out as above;
 * p_out (N x M(l) double, may be NULL) receives the nodal solution at the
 * unknowns, M(l) = mls2mc_ctx_n_unknowns(ctx, l).  Without p_out the FP64
 * solvers never store the solution (G is gathered from the CG search
 * directions), so a call with p_out streams one more vector per iteration;
 * G agrees between the two to rounding (same iterations).                  */
int mls2mc_forward_field(mls2mc_ctx* ctx, int l, int64_t N, const double* kappa,
                         double* G_out, double* p_out, int8_t* status_out,
                         int32_t* iters_out, void* stream);

/* Fused forward over many items (e.g. independent sampler instances and
 * levels): for each item, G_out = G_l(theta) as in mls2mc_forward, and
 * phi_out = Phi (Sec. 2.1 potential) when y is given.  All items run in one
 * grouped KL GEMM launch and one persistent solver launch over a device
 * work list (finest level first), cut into several such pairs only when
 * the coefficient buffer would exceed 8 GiB.  items is a host array.        */
typedef struct {
    int l;                /* level, within [l_min, l_max] of the context         */
    int64_t N;            /* particles                                            */
    const double* theta;  /* N x K                                                */
    double* G_out;        /* N x N_obs                                            */
    const double* y;      /* N_obs data for the fused potential, or NULL          */
    double* phi_out;      /* N, or NULL (needs y)                                 */
    int8_t* status_out;   /* N, or NULL                                           */
    int32_t* iters_out;   /* N, or NULL                                           */
} mls2mc_forward_item;
int mls2mc_forward_batch(mls2mc_ctx* ctx, int n_items, const mls2mc_forward_item* items,
                         void* stream);

/* Potential (Sec. 2.1): phi_out[q] = 1/2 sum_o ((y_o - G[q,o]) / sigma_n)^2.
 * G: N x N_obs, y: N_obs, phi_out: N (all double, device).                 */
int mls2mc_loglik(mls2mc_ctx* ctx, int64_t N, const double* G, const double* y,
                  double* phi_out, void* stream);

/* Adaptive step (Sec. 3.4, the argmin of (ESS - tau_ESS)^2 over the next
 * inverse temperature; tempering Sec. 3.1, bridging Sec. 3.2 and 4.1).
 * Incremental log-weights lw_j(t) = -t * scale * d_j with t = next - cur:
 * tempering: d = Phi_l, scale = 1, cur = beta; bridging: d = Phi_{l+1} -
 * Phi_l, scale = beta, cur = zeta.  ESS(t) = (sum e^lw)^2 / sum e^{2 lw}.
 * The chosen t is 1 - cur if ESS(1 - cur) >= tau_ess, else min(eps, 1-cur)
 * if ESS there is <= tau_ess, else the result of 64 bisection steps keeping
 * ESS(lo) >= tau_ess > ESS(hi) (lo returned).
 * Outputs (device): out3 = {next, dlogZ, ess} (3 doubles; next is exactly
 * 1.0 at the right end; dlogZ = LSE(lw) - log N); logw_out (N, may be NULL);
 * w_out (N, normalised weights exp(lw - LSE), may be NULL).
 * d: N doubles, finite (a non-finite entry gives next = NaN in out3).
 * Requires 0 <= cur < 1, eps > 0, 1 <= N <= 2^26.                          */
int mls2mc_next_step(mls2mc_ctx* ctx, int64_t N, const double* d, double scale, double cur,
                     double tau_ess, double eps, double* out3, double* logw_out,
                     double* w_out, void* stream);

/* Look-ahead statistic of the level-update test (Sec. 4.4): for the
 * weights w_j = exp(-scale d_j) on the N entries of d (the first J_tilde
 * particles, d = Phi_{l+1} - Phi_l, scale = beta, i.e. one bridging step
 * from zeta = 0 to 1), out2[0] = ESS = (sum w)^2 / sum w^2 and out2[1] =
 * cv^2 = N / ESS - 1, the squared coefficient of variation of the weights
 * with the population variance.  d: N doubles (device); out2: 2 doubles
 * (device).  A non-finite d_j gives NaN in both outputs.  Requires
 * 1 <= N <= 2^26 and scale >= 0.                                           */
int mls2mc_cv_lu(mls2mc_ctx* ctx, int64_t N, const double* d, double scale, double* out2, void* stream);

/* ---- update-scheme decision (host function, no device work) ---- */
#define MLS2MC_DECIDE_ITU 0     /* tempering update                        */
#define MLS2MC_DECIDE_LU 1      /* level update                            */
#define MLS2MC_DECIDE_DONE 2    /* finished: stop                          */
#define MLS2MC_DECIDE_NEED_CV 3 /* cv_lu is needed: compute it, call again */

/* The next update of the final update scheme (Sec. 4.4) and of the scheme
 * with an adaptive maximum level (Sec. 4.5), as mls2mc_run takes it.
 * beta: current inverse temperature; l, l_max: current and finest level;
 * prev_lu: 1 if the previous update was a level update or there was none
 * yet (the first update is a tempering update), else 0; scheme:
 * MLS2MC_SCHEME_MLS2MC or MLS2MC_SCHEME_MLB (multilevel bridging: tempering
 * up to beta = 1, then only level updates); cv_lu: coefficient of variation
 * of the level-update weights exp(-beta (Phi_{l+1} - Phi_l)) on the
 * look-ahead particles (mls2mc_cv_lu gives its square), or a negative value
 * when not computed; tau_lu: level-update threshold; tau_min:
 * the adaptive maximum level's threshold (0: off).
 * Rules: at beta = 1 and l = l_max: DONE.  At beta = 1: with tau_min > 0,
 * DONE when cv_lu < tau_min; otherwise LU.  Below beta = 1: ITU for
 * multilevel bridging, at l = l_max, or after a level update; otherwise LU
 * when cv_lu >= tau_lu, else ITU.  Returns NEED_CV when a rule needs cv_lu
 * and it is negative; -1 on bad arguments (l > l_max, beta outside [0, 1],
 * unknown scheme).                                                        */
int mls2mc_decide(double beta, int l, int l_max, int prev_lu, int scheme, double cv_lu, double tau_lu,
                  double tau_min);

/* Multinomial resampling (Sec. 2.4) with an exact integer CDF: weights are
 * scaled by the power of two that brings max w into [1/2,1), quantised to
 * q_j = floor(w_j 2^(62 - ceil(log2 N))), prefix-summed in uint64; for each
 * uniform u_i, t_i = floor(u_i 2^53 * C_N / 2^53) and anc[i] = min{j :
 * C_j > t_i}.  Bit-exact for given (w, u).  w: N doubles >= 0, not all
 * zero, any scale; u: N doubles in [0,1), multiples of 2^-53; anc_out: N
 * int32.  1 <= N <= 2^26.  Invalid weights give anc = -1 for every i.       */
int mls2mc_resample(mls2mc_ctx* ctx, int64_t N, const double* w, const double* u,
                    int32_t* anc_out, void* stream);

/* mls2mc_resample for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernel and the same ancestors for the same (w, u),
 * with the prefix sums in a static array the library holds on each GPU
 * (8 MiB, kept until the process ends) instead of context scratch; no
 * context is needed.  N <= 2^20 (EINVAL beyond, with a message).  It calls
 * no allocating routine (the array's address is looked up once per device,
 * on the first call there).  All calls on one GPU share the array: calls
 * that overlap in time on that GPU (on different streams or threads) race. */
int mls2mc_resample_noalloc(int64_t N, const double* w, const double* u, int32_t* anc_out,
                            void* stream);

/* Gather rows by ancestor: dst[i, :] = src[anc[i], :] for i < N, ncols
 * doubles per row; src has n_src rows; an ancestor outside [0, n_src) gives
 * a row of NaN.  src and dst must not overlap.                             */
int mls2mc_gather(mls2mc_ctx* ctx, int64_t N, int64_t ncols, const int32_t* anc,
                  int64_t n_src, const double* src, double* dst, void* stream);

/* One Metropolis-Hastings step (Markov move of Sec. 2.4) for the target
 * exp(-Psi) times the N(0, I) prior, Psi = beta [(1 - zeta) Phi_{l_lo} +
 * zeta Phi_{l_hi}].  Tempering: l_lo == l_hi (zeta ignored).  Bridging:
 * l_hi = l_lo + 1; the coarse level is evaluated only while zeta < 1.
 * kernel MLS2MC_KERNEL_PCN (pCN, cited in Secs. 1 and 5):
 *   theta' = sqrt(1 - s^2) theta + s xi;  accept iff log u < -(Psi' - Psi)
 *   (0 < s <= 1).
 * kernel MLS2MC_KERNEL_RWM (the random walk of the paper's Sec. 5 runs, whose
 * proposal covariance is 2.38^2 / K times the identity: pass s = 2.38 /
 * sqrt(K)):
 *   theta' = theta + s xi;  accept iff log u < -(Psi' + |theta'|^2 / 2 -
 *   Psi - |theta|^2 / 2)   (0 < s <= 10).
 * In/out state (device, double): theta N x K, G_lo / G_hi N x N_obs,
 * phi_lo / phi_hi N (caches of the current state; G_hi/phi_hi may be NULL
 * for tempering).  y: N_obs data.  xi: N x K normals; u: N uniforms in
 * (0,1).  accepted_out: N uint8 (may be NULL).  A proposal whose solve
 * fails (status != 0) is rejected.                                         */
/* Linear test model (the linear-Gaussian setting of Sec. 2.1, where every
 * tempered (Sec. 3.1) and bridged (Sec. 3.2) posterior is Gaussian in closed
 * form): after this call the forward map of level l is
 *   G_l(theta) = (A + 2^{-2l} E) theta
 * in every single-instance entry point that evaluates G (mls2mc_forward,
 * mls2mc_pcn_step, mls2mc_pcn_step_da, mls2mc_run), in place of the PDE;
 * solver status and iteration outputs read 0.  A, E: host arrays of
 * N_obs x K doubles (row-major), copied.  A = E = NULL restores the PDE.
 * mls2mc_forward_field, mls2mc_forward_batch and mls2mc_run_batch return
 * EINVAL while it is set.  For testing the sampler; synchronous.         */
int mls2mc_set_linear_model(mls2mc_ctx* ctx, const double* A, const double* E);

/* Linear surrogate for the delayed-acceptance first stage (the two-stage
 * Metropolis-Hastings screen of mls2mc_pcn_step_da): after this call the
 * surrogate's prediction is G~(theta) = S theta in mls2mc_surrogate_predict,
 * mls2mc_pcn_step_da and mls2mc_run, in place of the network, and no network
 * is needed (mls2mc_surrogate_init may be skipped).  In mls2mc_run with
 * surrogate on, the first stage then screens every pCN move from level
 * sur_da_min_level on (which may equal l_min), with no collection of
 * training pairs and no training.  S: host array of N_obs x K doubles
 * (row-major), copied; NULL restores the network.  With a linear model
 * (mls2mc_set_linear_model) the whole delayed-acceptance run is then fixed
 * by the paper's definitions and the random streams, which the tests
 * compare stage by stage with the oracle's sampler.  For testing;
 * synchronous.                                                             */
int mls2mc_set_linear_surrogate(mls2mc_ctx* ctx, const double* S);

#define MLS2MC_KERNEL_PCN 0
#define MLS2MC_KERNEL_RWM 1

typedef struct {
    int l_lo, l_hi;
    double beta, zeta;
    double s;          /* step size (see above)                            */
    int kernel;        /* MLS2MC_KERNEL_PCN or MLS2MC_KERNEL_RWM           */
} mls2mc_stage;

int mls2mc_pcn_step(mls2mc_ctx* ctx, const mls2mc_stage* st, int64_t N, double* theta,
                    double* G_lo, double* G_hi, double* phi_lo, double* phi_hi,
                    const double* y, const double* xi, const double* u,
                    uint8_t* accepted_out, void* stream);

/* ---- learned surrogate theta -> G(theta) (MLP K -> H -> H -> N_obs) ---- */
/* The network has two hidden layers of width `hidden` with erf-GELU
 * activations; matrix products run as BF16 MFMA with FP32 accumulation,
 * master weights and Adam moments are FP32.  Parameter layout (FP32):
 * W1[H x K], b1[H], W2[H x H], b2[H], W3[N_obs x H], b3[N_obs] (row-major,
 * out x in).  Inputs and outputs are standardised with the mean and standard
 * deviation of the training pairs (per component) once training has run.  */
/* (Re)create the surrogate: He-initialised weights (Philox normals from
 * `seed`), zero biases, an empty ring of `capacity` training pairs.
 * hidden: multiple of 16 in [16, 1024].  Synchronous.                      */
int mls2mc_surrogate_init(mls2mc_ctx* ctx, int hidden, int64_t capacity, uint64_t seed,
                          void* stream);
int mls2mc_surrogate_n_params(const mls2mc_ctx* ctx);
int64_t mls2mc_surrogate_n_pairs(const mls2mc_ctx* ctx);
/* copy FP32 parameters in / out (device arrays of n_params floats)         */
int mls2mc_surrogate_set_params(mls2mc_ctx* ctx, const float* params, void* stream);
int mls2mc_surrogate_get_params(mls2mc_ctx* ctx, float* params, void* stream);
/* append n pairs (theta: n x K, G: n x N_obs, device doubles) to the ring;
 * the ring keeps the most recent `capacity` pairs.                          */
int mls2mc_surrogate_add_pairs(mls2mc_ctx* ctx, int64_t n, const double* theta, const double* G,
                               void* stream);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the mean over batch and outputs
 * of (net(x) - t)^2 / 2 with standardised x, t; `epochs` passes over a host-
 * shuffled permutation (seeded) in minibatches of `batch`.  loss_out (host,
 * may be NULL) receives the last minibatch loss of each epoch.  Synchronous
 * at epoch ends.  Needs at least `batch` pairs.                            */
int mls2mc_surrogate_train(mls2mc_ctx* ctx, int epochs, int batch, double lr, uint64_t seed,
                           float* loss_out, void* stream);
/* G_out[N x N_obs] = surrogate(theta[N x K]) in the units of G.             */
int mls2mc_surrogate_predict(mls2mc_ctx* ctx, int64_t N, const double* theta, double* G_out,
                             void* stream);
/* Loss and its gradient for raw (unstandardised) inputs x[B x K] and targets
 * t[B x N_obs] (device doubles): loss_out (1 float), grad_out (n_params
 * floats), both device.  For gradient checks.                              */
int mls2mc_surrogate_loss_grad(mls2mc_ctx* ctx, int64_t B, const double* x, const double* target,
                               float* loss_out, float* grad_out, void* stream);
/* Delayed-acceptance pCN step (two-stage Metropolis-Hastings, Christen and
 * Fox 2005) for the same target as mls2mc_pcn_step.  Stage 1 accepts iff
 * log u1 < -(Psi~' - Psi~) with Psi~ = beta Phi(surrogate(theta)); only the
 * stage-1 survivors are solved with the FEM forward (compacted on the
 * device, no host synchronisation); stage 2 accepts iff log u2 < -(Psi' -
 * Psi) + (Psi~' - Psi~).  The chain is exact for any surrogate.
 * accepted_out (N uint8) and stage1_out (N uint8, may be NULL) receive the
 * outcomes; n_solved_lo / n_solved_hi (device int64, may be NULL) are
 * incremented by the number of solves done on l_lo / l_hi.                 */
int mls2mc_pcn_step_da(mls2mc_ctx* ctx, const mls2mc_stage* st, int64_t N, double* theta,
                       double* G_lo, double* G_hi, double* phi_lo, double* phi_hi,
                       const double* y, const double* xi, const double* u1, const double* u2,
                       uint8_t* accepted_out, uint8_t* stage1_out, int64_t* n_solved_lo,
                       int64_t* n_solved_hi, void* stream);

/* ---- the whole MLS^2MC sampler (Sec. 4, update scheme of Sec. 4.4) ---- */
typedef struct {
    int64_t J;          /* particles, 1 <= J <= 2^26                        */
    int64_t J_tilde;    /* look-ahead particles for cv^LU, 1..J (0 = min(100,J)) */
    double tau_star;    /* target cv: tau_ESS = J / (1 + tau_star^2)         */
    double tau_lu;      /* level-update threshold (0 = tau_star)             */
    double eps;         /* minimum temperature increment (0 = 1e-6)          */
    int n_mcmc;         /* pCN steps per stage                              */
    double s_pcn;       /* pCN step size                                    */
    uint64_t seed;      /* Philox key                                       */
    int max_stages;     /* safety cap (0 = 4000)                            */
    /* learned surrogate with delayed acceptance (0 = off).  Pairs (theta',
     * G_l(theta')) of the pCN proposals of tempering stages on levels <=
     * sur_collect_max_level go into the ring; the network is trained once on
     * reaching level sur_da_min_level and every pCN step on levels >= it is
     * a delayed-acceptance step (second-stage uniforms: Philox stream 6).   */
    int surrogate;
    int sur_collect_max_level;
    int sur_da_min_level;
    int64_t sur_pairs;  /* ring capacity (0 = 20480)                        */
    int sur_epochs;     /* 0 = 15                                           */
    int sur_hidden;     /* 0 = 256                                          */
    int sur_batch;      /* 0 = 256                                          */
    double sur_lr;      /* 0 = 1e-3                                         */
    /* optional pCN step adaptation, an extension that the paper does not
     * use (0 = fixed s_pcn): after each stage s <- clamp(s exp(2 (a -
     * 0.25)), 0.005, 1) with a the stage's acceptance rate.               */
    int s_adapt;
    /* update scheme: MLS2MC_SCHEME_MLS2MC, the adaptive scheme of Sec. 4.4,
     * or MLS2MC_SCHEME_MLB, multilevel bridging (Example in Sec. 4): temper
     * on l_min up to beta = 1, then bridge level by level.                 */
    int scheme;
    /* adaptive maximum level (the modified scheme u' of Sec. 4.5; 0 = off):
     * at beta = 1 and l < l_max, cv^LU is estimated on the first J_tilde
     * particles and the run stops at level l when cv^LU < tau_min (the
     * paper uses 0.001); otherwise the look-ahead solves are reused.      */
    double tau_min;
    int kernel;         /* MLS2MC_KERNEL_PCN (default) or MLS2MC_KERNEL_RWM */
} mls2mc_run_config;

#define MLS2MC_SCHEME_MLS2MC 0
#define MLS2MC_SCHEME_MLB 1

typedef struct {
    int n_stages;
    int final_level;
    double final_beta;
    double log_Z;          /* sum over reweightings of LSE(lw) - log J       */
    int64_t solves[16];    /* forward solves per level                       */
    int64_t accepted, proposed;
    int64_t iters_total;   /* PCG iterations summed over all solves          */
    int64_t not_converged; /* solves reported with status != 0               */
    double seconds;        /* wall time of the run (host clock)              */
    int64_t stage1_passed; /* delayed acceptance: proposals solved with FEM  */
    int64_t da_proposed;   /* delayed acceptance: proposals screened         */
    double sur_train_seconds;
    double sur_final_loss;
    int64_t graphs_launched; /* mls2mc_run_batch: HIP graphs launched        */
    /* optional per-stage log (host arrays of max_stage_log entries, or NULL).
     * stage types: 0 tempering, 1 tempering after a discarded look-ahead,
     * 2 first bridging sub-step of a level update chosen by the look-ahead,
     * 3 first bridging sub-step of a level update forced at beta = 1,
     * 4 later bridging sub-step                                             */
    int max_stage_log;
    int* stage_type;
    int* stage_level;
    double* stage_beta;
    double* stage_zeta;
    double* stage_ess;
    double* stage_acc_rate;
    /* delayed acceptance: error of the surrogate against the FEM solve that
     * judges each stage-1 survivor, e = ||G~(theta') - G(theta')||_2 / sigma_n
     * with G on the finer level of the move: mean and max over the run, the
     * number of survivors, and per stage (host arrays of max_stage_log
     * entries, or NULL; NaN for stages without delayed acceptance)         */
    double sur_err_mean, sur_err_max;
    int64_t sur_err_count;
    double* stage_sur_err_mean;
    double* stage_sur_err_max;
} mls2mc_run_result;

/* Run MLS^2MC from the prior to beta = 1 on level l_max.  y: N_obs data
 * (device).  theta_out: J x K final particles (device, equally weighted).
 * Synchronous (returns when done).  Random streams (Philox4x32-10, counter
 * = {index, sub-step, stage, stream}, key = seed): 0 prior draw, 3
 * resampling uniforms, 4 pCN normals, 5 pCN uniforms.                      */
int mls2mc_run(mls2mc_ctx* ctx, const mls2mc_run_config* cfg, const double* y,
               double* theta_out, mls2mc_run_result* res, void* stream);

/* Many independent MLS^2MC instances (own data, seed, particle count and
 * finest level; shared problem of the context) in lock-step rounds: each
 * round every active instance performs one SMC sub-step.  The forward
 * solves of a phase, across all instances and levels, run as one fused
 * work-list launch, and with use_graphs != 0 the mutation phase of each round
 * (all pCN steps of all instances) is captured as a HIP graph and launched
 * once.  Each instance draws the Philox streams of mls2mc_run with its own
 * seed.  cfg supplies the shared settings (J and seed are per instance;
 * the surrogate fields must be 0).  res: n_inst results.  stream may be NULL
 * (a private stream is used; capture needs a non-default stream).
 * Synchronous.                                                             */
typedef struct {
    int64_t J;          /* particles                                        */
    int l_max;          /* finest level of this instance                    */
    const double* y;    /* N_obs data (device)                              */
    uint64_t seed;      /* Philox key                                       */
    double* theta_out;  /* J x K final particles (device)                   */
} mls2mc_instance;
int mls2mc_run_batch(mls2mc_ctx* ctx, const mls2mc_run_config* cfg, int n_inst,
                     const mls2mc_instance* inst, mls2mc_run_result* res, int use_graphs,
                     void* stream);

/* Philox4x32-10 uniforms/normals on the device, the same streams mls2mc_run
 * uses (6: second-stage uniforms of delayed acceptance): out[i] for idx = i, counter {idx, sub, stage, stream}.  normal = 0:
 * uniform in [0,1) (multiple of 2^-53); normal = 1: Box-Muller normal.      */
int mls2mc_philox_fill(mls2mc_ctx* ctx, uint64_t seed, uint32_t stream_id, uint32_t stage,
                       uint32_t sub, int64_t n, int normal, double* out, void* stream);

/* ---- launch shape of the persistent solver ---- */
/* Autotune the solver for level l on N prior draws: every candidate
 * (persistent workgroups = w x CUs capped at N; block size; V-cycle
 * Gauss-Seidel sweeps per side nu in {1,2}; LDS residency of the multigrid
 * hierarchy and of the finest level's arrays, for the flow cell of the
 * coarse levels only: none, 64 KiB, 80 KiB or the device's LDS per
 * workgroup less 1 KiB) solves the batch to the context's
 * tolerance, is timed with HIP events (best of 3), and the fastest is kept
 * in the context for level l.  best_ms (host, may be NULL) receives its
 * time.  Synchronous; allocates its own temporary buffers.                 */
int mls2mc_autotune(mls2mc_ctx* ctx, int l, int64_t N, double* best_ms, void* stream);
/* Read / set the solver schedule of level l (grid 0, block 0, nu 0 or
 * lds_bytes 0 = built-in default; lds_bytes -1 = no LDS residency, else
 * the per-workgroup LDS budget in bytes, at most the device's LDS per
 * workgroup less 1 KiB; 160 KiB on gfx950), e.g. to restore tuned
 * schedules cached by the caller.                                          */
int mls2mc_get_launch(const mls2mc_ctx* ctx, int l, int* grid, int* block, int* nu, int* lds_bytes);
int mls2mc_set_launch(mls2mc_ctx* ctx, int l, int grid, int block, int nu, int lds_bytes);

/* ---- kernel-time instrumentation ---- */
/* When enabled, the library records a pair of HIP events on the launch
 * stream around every launch of the solver kernel and of the KL GEMM, and
 * accumulates the PCG iterations of the solved particles on the device.
 * enable = 1 clears the records and starts; enable = 0 stops (records are
 * kept until the next enable = 1).                                         */
#define MLS2MC_PROF_SOLVE 0 /* multigrid-PCG solver kernel (incl. observation) */
#define MLS2MC_PROF_GEMM 1  /* KL field GEMM                                   */
typedef struct {
    int64_t launches; /* launches recorded                                 */
    double ms;        /* summed event-measured kernel durations            */
    int64_t items;    /* particles (solver) or field rows (GEMM)            */
    int64_t iters;    /* PCG iterations summed over particles (solver; MIXED:
                         inner iterations over all refinement sweeps)       */
} mls2mc_prof_entry;
int mls2mc_profile(mls2mc_ctx* ctx, int enable);
/* Totals for one kernel class and level (synchronizes the device).         */
int mls2mc_profile_read(mls2mc_ctx* ctx, int kclass, int l, mls2mc_prof_entry* out);

#ifdef __cplusplus
}
#endif
#endif
