/*
 * CPU FP64 oracle for Multilevel Sequential^2 Monte Carlo (Latz, Papaioannou,
 * Ullmann, "Multilevel Sequential^2 Monte Carlo for Bayesian Inverse
 * Problems", J. Comp. Phys.).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU path is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code, no
 * header and no table with the HIP library; the two never include or link
 * each other.
 *
 * Every routine works in IEEE double precision (the paper fixes no
 * precision).  Arrays are caller-owned, row-major and particle-major.
 * Functions return 0 on success and a negative value on bad arguments
 * (-1), allocation failure (-2) or a numerically singular situation (-3).
 *
 * Parity status of each part (what pins it lives in tests/):
 *   philox          pinned: published known-answer vectors.
 *   kl modes/basis  pinned: Nystrom eigenvalues, orthonormality, eigen
 *                   equation residual, boundary conditions, trace.
 *   assembly/solve  pinned: nodal-exact manufactured solution, O(h^2)
 *                   convergence, torsion series, sine-mode eigenpairs,
 *                   symmetry/SPD, dense-solve cross-check on tiny meshes.
 *   observation     pinned: nodal points, exactness on linear fields.
 *   next_step       pinned: Kish identity, monotonicity, limits.
 *   resample        pinned: brute force on exact rationals, chi^2.
 *   sampler         pinned: linear-Gaussian closed-form posterior/evidence,
 *                   solve-count identity, single-level special case.
 *   mlp             pinned: central finite differences.
 *   posterior on the PDE model: parity unpinned against truth (no closed
 *                   form); only GPU-vs-oracle agreement is checked.
 */
#ifndef MLS2MC_ORACLE_H
#define MLS2MC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), own implementation */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* uniform in [0,1), an exact multiple of 2^-53, from one Philox block     */
double orc_uniform(uint64_t seed, uint32_t stream, uint32_t stage, uint32_t sub, uint32_t idx);
/* standard normal by Box-Muller from one Philox block                     */
double orc_normal(uint64_t seed, uint32_t stream, uint32_t stage, uint32_t sub, uint32_t idx);

/* ---- Karhunen-Loeve expansion of the separable exponential covariance ---- */
/* 1-D: positive roots omega_n of (w^2-c^2) sin w - 2 c w cos w, c = 1/corr;
 * mu_n = 2c/(w^2+c^2).                                                     */
int orc_kl_roots_1d(int nmodes, double corr_len, double* omega, double* mu);
/* evaluate the normalised 1-D eigenfunction n (0-based) at t              */
double orc_kl_phi_1d(double omega, double corr_len, double t);
/* 2-D modes: first K of sigma2*mu_i*mu_j, descending, tie -> smaller i.   */
int orc_kl_modes_2d(int K, double sigma2, double corr_len,
                    double* lambda /*K*/, int* ix /*K*/, int* iy /*K*/,
                    double* omega_x /*K*/, double* omega_y /*K*/);
/* B[k*n_e + e] = sqrt(lambda_k) phi_k(centroid_e), n_e = 2*4^l            */
int orc_kl_basis(int l, int K, double sigma2, double corr_len, double* B);
/* a[N x n_e] = theta[N x K] * B[K x n_e]                                 */
int orc_kl_field(int l, int K, int64_t N, const double* B, const double* theta, double* a);

/* ---- mesh ---- */
/* centroid of element e on level l: x = (3i+2)/(3n) etc.                 */
void orc_centroid(int l, int e, double* x, double* y);

/* ---- FEM assembly and banded Cholesky solve ---- */
/* Assemble the stiffness matrix of -div(kappa grad p) with P1 elements
 * (generic per-triangle element matrices) in symmetric band storage:
 * band[u*(bw+1) + k] = A[u][u-k], k = 0..bw, bw = n (the triangle
 * connectivity half-bandwidth), M = (n-1)^2.                              */
int orc_assemble_band(int l, const double* kappa /*n_e*/, double* band);
/* dense copy of A, M x M (tiny meshes only)                               */
int orc_assemble_dense(int l, const double* kappa, double* A);
/* load b_u = int f phi_u with f == 1 (exact), or nodal quadrature h^2 f(x_u)
 * if f_nodal != NULL (f_nodal has one value per interior node).           */
int orc_load(int l, const double* f_nodal, double* b);
/* Solve A(kappa) p = b by banded Cholesky.  p: interior values, length M. */
int orc_solve(int l, const double* kappa, const double* b, double* p);

/* ---- observation, potential ---- */
/* observation points (a/(m+1), b/(m+1)), a,b = 1..m, o = (b-1)m+(a-1)     */
int orc_observe(int l, int m, const double* p_interior, double* G);
double orc_potential(int nobs, const double* G, const double* y, double sigma_n);

/* full forward map theta -> G for a batch (OpenMP over particles)         */
int orc_forward(int l, int K, double sigma2, double corr_len, int m,
                int64_t N, const double* theta, double* G, int nthreads);
/* forward map from a given kappa batch (N x n_e)                         */
int orc_forward_kappa(int l, int m, int64_t N, const double* kappa, double* G,
                      double* p_out /*N x M or NULL*/, int nthreads);

/* ---- adaptive SMC step: effective sample size and next temperature ---- */
double orc_ess(int64_t N, const double* d, double scale, double t);
int orc_next_step(int64_t N, const double* d, double scale, double cur,
                  double tau_ess, double eps, double* next, double* logw,
                  double* w, double* dlogZ, double* ess);

/* ---- multinomial resampling with an exact integer CDF ---- */
int orc_resample(int64_t N, const double* w, const double* u, int32_t* anc);

/* ---- pCN proposal and Metropolis-Hastings acceptance ---- */
/* Gaussian random-walk proposal theta' = theta + s xi                    */
void orc_rwm_propose(int64_t N, int K, double s, const double* theta, const double* xi,
                     double* theta_new);
void orc_pcn_propose(int64_t N, int K, double s, const double* theta,
                     const double* xi, double* theta_new);
/* returns 1 if accepted: log u < -(psi_new - psi_old)                     */
int orc_mh_accept(double psi_old, double psi_new, double u);

/* delayed acceptance (two-stage Metropolis-Hastings of Christen and Fox,
 * 2005) with a cheap approximation psis of the potential psi: stage 1
 * accepts iff log u1 < -(psis_new - psis_old); stage 2, reached only after
 * stage 1, accepts iff log u2 < -(psi_new - psi_old) + (psis_new -
 * psis_old).  Returns 1 if the move is accepted; *stage1 = stage-1 outcome. */
int orc_da_accept(double psi_old, double psi_new, double psis_old, double psis_new,
                  double u1, double u2, int* stage1);

/* Flow cell of Example 5.3 (Sec. 5): -div(kappa grad p) = 0, p = 0 at
 * x1 = 0, p = 1 at x1 = 1, no flow through x2 = 0 and x2 = 1, P1 elements
 * on the mesh of level l (generic per-triangle assembly over the unknown
 * nodes 1 <= i <= n-1, 0 <= j <= n, u = j (n-1) + (i-1), the value 1 of
 * the right edge moved to the right-hand side, banded Cholesky), observed
 * at (a/(m+1), b/(m+1)) by P1 interpolation of the nodal values, boundary
 * values included.  p_out (may be NULL): the unknowns' values.           */
int orc_flow_forward_kappa(int l, int m, int64_t N, const double* kappa, double* G, double* p_out,
                           int nthreads);

/* ---- the MLS^2MC sampler ---- */
enum { ORC_MODEL_PDE = 0, ORC_MODEL_LINEAR = 1, ORC_MODEL_FLOWCELL = 2 };

typedef struct {
    int model;          /* ORC_MODEL_PDE, ORC_MODEL_LINEAR or ORC_MODEL_FLOWCELL */
    int l_min, l_max;   /* level range (h = 2^-l)                            */
    int K;              /* parameter dimension                               */
    double sigma2, corr_len;
    int m;              /* observation grid side; N_obs = m*m (PDE model)    */
    int nobs;           /* observation count (linear model)                  */
    double sigma_n;     /* noise standard deviation                          */
    int64_t J;          /* particles                                         */
    int64_t J_tilde;    /* look-ahead particles for the level-update test    */
    double tau_ess;     /* ESS target (J/(1+tau*^2))                          */
    double tau_lu;      /* level-update threshold on cv                      */
    double eps;         /* minimum step of the temperature                   */
    int n_mcmc;         /* pCN steps per stage                               */
    double s_pcn;       /* pCN step size                                     */
    uint64_t seed;      /* random streams                                    */
    int max_stages;
    int nthreads;
    /* linear model G_l(theta) = (A + 2^{-2l} E) theta, each nobs x K       */
    const double* lin_A;
    const double* lin_E;
    /* delayed-acceptance pCN with the linear surrogate G~(theta) = S theta
     * (nobs x K, linear model only); NULL = plain pCN.  Uniforms of the
     * second stage come from stream 6.                                     */
    const double* da_S;
    /* optional pCN step adaptation (not in the paper; 0 = fixed s_pcn):
     * after each stage s <- clamp(s exp(2 (a - 0.25)), 0.005, 1), a the
     * stage's acceptance rate.                                             */
    int s_adapt;
    /* update scheme: 0 the adaptive scheme u of Sec. 4.4; 1 multilevel
     * bridging (the Sec. 4 example: temper on l_min to beta = 1, then
     * bridge level by level)                                               */
    int scheme;
    /* the modified scheme u' of Sec. 4.5 (0 = off): at beta = 1 and
     * l < l_max stop when cv^LU < tau_min                                  */
    double tau_min;
    /* Markov kernel: 0 pCN; 1 Gaussian random walk theta + s xi with the
     * N(0, I) prior ratio in the acceptance (the kernel of the Sec. 5 runs) */
    int kernel;
} orc_config;

typedef struct {
    int n_stages;
    double log_Z;
    int final_level;
    double final_beta;
    int64_t solves[16];     /* forward evaluations per level                */
    int64_t accepted, proposed;
    int64_t stage1_passed;  /* delayed acceptance: proposals past stage 1   */
    /* per stage: type, level, beta, zeta, ESS.  Types: 0 tempering update,
     * 1 tempering update after a discarded look-ahead, 2 first bridging
     * sub-step of a level update chosen by the look-ahead, 3 first bridging
     * sub-step of a level update forced at beta = 1, 4 later sub-step.     */
    int* stage_type;
    int* stage_level;
    double* stage_beta;
    double* stage_zeta;
    double* stage_ess;
    double* stage_step;     /* pCN step used in the stage's mutation          */
    double* stage_acc_rate; /* accepted / (J n_mcmc) in the stage's mutation  */
    int max_stage_log;
} orc_result;

/* y: data (nobs); theta_out: final particles J x K (caller-owned).        */
int orc_run_sampler(const orc_config* cfg, const double* y, double* theta_out,
                    orc_result* res);

/* ---- MLP surrogate reference: 2 hidden layers, erf-GELU, MSE ---- */
/* params: W1[H1 x D], b1[H1], W2[H2 x H1], b2[H2], W3[O x H2], b3[O].
 * forward for a batch; loss = mean over batch and outputs of (out-t)^2/2.
 * grad (same layout as params) is d loss / d params.                      */
int orc_mlp_forward(int D, int H1, int H2, int O, const double* params,
                    int64_t B, const double* x, double* out);
int orc_mlp_loss_grad(int D, int H1, int H2, int O, const double* params,
                      int64_t B, const double* x, const double* target,
                      double* loss, double* grad);

#ifdef __cplusplus
}
#endif
#endif
