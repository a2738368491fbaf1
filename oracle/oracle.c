/*
 * CPU FP64 oracle for Multilevel Sequential^2 Monte Carlo.
 *
 * TEST INFRASTRUCTURE ONLY: slow, plain and written for reading against the
 * paper, not for speed.  It shares nothing with the HIP library.  See
 * oracle.h for the parity status of each part.
 *
 * Citations name the paper's sections and equations:
 *   problem statement, potential and evidence ............ Sec. 2.1
 *   particle approximation ................................ Sec. 2.2
 *   importance sampling with self-normalised weights ....... Sec. 2.3
 *   SMC: reweight, resample, Markov move ................... Sec. 2.4
 *   tempering ............................................. Sec. 3.1
 *   bridging .............................................. Sec. 3.2
 *   ESS / coefficient of variation, next-temperature argmin  Sec. 3.4
 *   MLS^2MC updates (ITU, LU with bridging sub-steps) ...... Sec. 4.1
 *   solve-count model ...................................... Sec. 4.2, Prop. 4.4
 *   look-ahead cv^LU test and final update scheme ......... Sec. 4.4
 *   forward model: -div(kappa grad p) = f, kappa = exp(theta),
 *   truncated KL expansion, P1 elements, point observations  Sec. 5
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ESING (-3)

/* ======================================================================
 * Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11): ten rounds of the multiply-xor bijection with the
 * Weyl key schedule.
 * ==================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void orc_block(uint64_t seed, uint32_t stream, uint32_t stage, uint32_t sub,
                      uint32_t idx, uint32_t out[4])
{
    uint32_t ctr[4] = {idx, sub, stage, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* 53 random bits -> exact multiple of 2^-53 in [0,1) */
static double orc_u53(uint32_t hi, uint32_t lo)
{
    uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
    return (double)v * 0x1.0p-53;
}

double orc_uniform(uint64_t seed, uint32_t stream, uint32_t stage, uint32_t sub, uint32_t idx)
{
    uint32_t o[4];
    orc_block(seed, stream, stage, sub, idx, o);
    return orc_u53(o[0], o[1]);
}

double orc_normal(uint64_t seed, uint32_t stream, uint32_t stage, uint32_t sub, uint32_t idx)
{
    uint32_t o[4];
    orc_block(seed, stream, stage, sub, idx, o);
    double u1 = 1.0 - orc_u53(o[0], o[1]); /* (0,1] */
    double u2 = orc_u53(o[2], o[3]);       /* [0,1) */
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* ======================================================================
 * Karhunen-Loeve expansion (Sec. 5, truncated KL expansion of the prior
 * field; the covariance here is the separable exponential
 * C(x,x') = sigma2 exp(-|x1-x1'|/corr) exp(-|x2-x2'|/corr)).
 *
 * 1-D integral eigenproblem on [0,1] with c = 1/corr: eigenfunctions
 * A cos(wt) + B sin(wt) with phi'(0) = c phi(0), phi'(1) = -c phi(1), which
 * gives B/A = c/w and (w^2 - c^2) sin w - 2 c w cos w = 0; eigenvalue
 * mu = 2c / (w^2 + c^2).  The n-th positive root lies in ((n-1)pi, n pi).
 * ==================================================================== */
static double orc_kl_g(double w, double c)
{
    return (w * w - c * c) * sin(w) - 2.0 * c * w * cos(w);
}

int orc_kl_roots_1d(int nmodes, double corr_len, double* omega, double* mu)
{
    if (nmodes <= 0 || !(corr_len > 0)) return ORC_EINVAL;
    double c = 1.0 / corr_len;
    for (int n = 1; n <= nmodes; ++n) {
        double lo = (n - 1) * M_PI, hi = n * M_PI;
        if (n == 1) lo = 1e-300;
        double glo = orc_kl_g(lo, c);
        if (n == 1) glo = -1.0; /* g(w) ~ w (w^2 - c^2 - 2c) < 0 near 0 */
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            double gm = orc_kl_g(mid, c);
            if ((gm < 0) == (glo < 0)) { lo = mid; glo = gm; }
            else hi = mid;
        }
        double w = 0.5 * (lo + hi);
        omega[n - 1] = w;
        mu[n - 1] = 2.0 * c / (w * w + c * c);
    }
    return 0;
}

double orc_kl_phi_1d(double omega, double corr_len, double t)
{
    double c = 1.0 / corr_len;
    double A = omega / c, B = 1.0;
    double s2w = sin(2.0 * omega), sw = sin(omega);
    double nrm2 = A * A * (0.5 + s2w / (4.0 * omega)) + B * B * (0.5 - s2w / (4.0 * omega))
                + A * B * sw * sw / omega;
    return (A * cos(omega * t) + B * sin(omega * t)) / sqrt(nrm2);
}

typedef struct { double lam; int i, j; } orc_mode;

static int orc_mode_cmp(const void* pa, const void* pb)
{
    const orc_mode* a = (const orc_mode*)pa;
    const orc_mode* b = (const orc_mode*)pb;
    if (a->lam > b->lam) return -1;
    if (a->lam < b->lam) return 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    return a->j < b->j ? -1 : (a->j > b->j);
}

int orc_kl_modes_2d(int K, double sigma2, double corr_len, double* lambda, int* ix, int* iy,
                    double* omega_x, double* omega_y)
{
    if (K <= 0) return ORC_EINVAL;
    int nm = K;
    double* om = (double*)malloc(sizeof(double) * nm);
    double* mu = (double*)malloc(sizeof(double) * nm);
    orc_mode* all = (orc_mode*)malloc(sizeof(orc_mode) * (size_t)nm * nm);
    if (!om || !mu || !all) { free(om); free(mu); free(all); return ORC_ENOMEM; }
    int rc = orc_kl_roots_1d(nm, corr_len, om, mu);
    if (rc == 0) {
        for (int i = 0; i < nm; ++i)
            for (int j = 0; j < nm; ++j) {
                orc_mode* md = &all[(size_t)i * nm + j];
                md->lam = sigma2 * (mu[i] * mu[j]); /* exact (i,j)/(j,i) ties */
                md->i = i; md->j = j;
            }
        qsort(all, (size_t)nm * nm, sizeof(orc_mode), orc_mode_cmp);
        for (int k = 0; k < K; ++k) {
            lambda[k] = all[k].lam;
            ix[k] = all[k].i; iy[k] = all[k].j;
            omega_x[k] = om[all[k].i]; omega_y[k] = om[all[k].j];
        }
    }
    free(om); free(mu); free(all);
    return rc;
}

/* ======================================================================
 * Mesh (Sec. 5: P1 elements on uniform meshes with 2 n^2 triangles).
 * n = 2^l, nodes (i h, j h).  Cell (i,j) is cut by the diagonal from (i,j)
 * to (i+1,j+1); element 2(jn+i) is the lower triangle
 * {(i,j),(i+1,j),(i+1,j+1)}, element 2(jn+i)+1 the upper triangle
 * {(i,j),(i+1,j+1),(i,j+1)}.  Interior node (i,j), 1<=i,j<=n-1, has
 * unknown index (j-1)(n-1)+(i-1).
 * ==================================================================== */
void orc_centroid(int l, int e, double* x, double* y)
{
    int n = 1 << l;
    int cell = e >> 1, t = e & 1;
    int i = cell % n, j = cell / n;
    if (t == 0) { *x = (double)(3 * i + 2) / (double)(3 * n); *y = (double)(3 * j + 1) / (double)(3 * n); }
    else        { *x = (double)(3 * i + 1) / (double)(3 * n); *y = (double)(3 * j + 2) / (double)(3 * n); }
}

static void orc_tri_nodes(int n, int e, int vi[3], int vj[3])
{
    int cell = e >> 1, t = e & 1;
    int i = cell % n, j = cell / n;
    if (t == 0) { vi[0] = i; vj[0] = j; vi[1] = i + 1; vj[1] = j; vi[2] = i + 1; vj[2] = j + 1; }
    else        { vi[0] = i; vj[0] = j; vi[1] = i + 1; vj[1] = j + 1; vi[2] = i; vj[2] = j + 1; }
}

int orc_kl_basis(int l, int K, double sigma2, double corr_len, double* B)
{
    if (l < 1 || l > 12 || K <= 0) return ORC_EINVAL;
    double* lam = (double*)malloc(sizeof(double) * K);
    int* ix = (int*)malloc(sizeof(int) * K);
    int* iy = (int*)malloc(sizeof(int) * K);
    double* ox = (double*)malloc(sizeof(double) * K);
    double* oy = (double*)malloc(sizeof(double) * K);
    if (!lam || !ix || !iy || !ox || !oy) { free(lam); free(ix); free(iy); free(ox); free(oy); return ORC_ENOMEM; }
    int rc = orc_kl_modes_2d(K, sigma2, corr_len, lam, ix, iy, ox, oy);
    if (rc == 0) {
        int n = 1 << l, ne = 2 * n * n;
        for (int k = 0; k < K; ++k) {
            double sl = sqrt(lam[k]);
            for (int e = 0; e < ne; ++e) {
                double x, y;
                orc_centroid(l, e, &x, &y);
                B[(size_t)k * ne + e] = sl * orc_kl_phi_1d(ox[k], corr_len, x) * orc_kl_phi_1d(oy[k], corr_len, y);
            }
        }
    }
    free(lam); free(ix); free(iy); free(ox); free(oy);
    return rc;
}

int orc_kl_field(int l, int K, int64_t N, const double* B, const double* theta, double* a)
{
    int n = 1 << l, ne = 2 * n * n;
    for (int64_t p = 0; p < N; ++p)
        for (int e = 0; e < ne; ++e) {
            double s = 0.0;
            for (int k = 0; k < K; ++k) s += theta[p * K + k] * B[(size_t)k * ne + e];
            a[p * ne + e] = s;
        }
    return 0;
}

/* ======================================================================
 * P1 stiffness matrix, generic per-triangle assembly:
 * K^T_ab = kappa_T |T| grad(phi_a) . grad(phi_b), Dirichlet nodes dropped.
 * ==================================================================== */
static int orc_unknown(int n, int i, int j)
{
    if (i < 1 || j < 1 || i > n - 1 || j > n - 1) return -1;
    return (j - 1) * (n - 1) + (i - 1);
}

static void orc_local_stiffness(int n, int e, double kappa, int gu[3], double Kl[3][3])
{
    int vi[3], vj[3];
    double h = 1.0 / n;
    orc_tri_nodes(n, e, vi, vj);
    double x[3], y[3];
    for (int a = 0; a < 3; ++a) { x[a] = vi[a] * h; y[a] = vj[a] * h; gu[a] = orc_unknown(n, vi[a], vj[a]); }
    double det = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
    double area = 0.5 * fabs(det);
    double gx[3], gy[3];
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        gx[a] = (y[b] - y[c]) / det;
        gy[a] = (x[c] - x[b]) / det;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Kl[a][b] = kappa * area * (gx[a] * gx[b] + gy[a] * gy[b]);
}

int orc_assemble_band(int l, const double* kappa, double* band)
{
    if (l < 1 || l > 12) return ORC_EINVAL;
    int n = 1 << l, ne = 2 * n * n, M = (n - 1) * (n - 1), bw = n;
    memset(band, 0, sizeof(double) * (size_t)M * (bw + 1));
    for (int e = 0; e < ne; ++e) {
        int gu[3];
        double Kl[3][3];
        orc_local_stiffness(n, e, kappa[e], gu, Kl);
        for (int a = 0; a < 3; ++a) {
            if (gu[a] < 0) continue;
            for (int b = 0; b < 3; ++b) {
                if (gu[b] < 0 || gu[b] > gu[a]) continue;
                int k = gu[a] - gu[b];
                if (k > bw) return ORC_EINVAL;
                band[(size_t)gu[a] * (bw + 1) + k] += Kl[a][b];
            }
        }
    }
    return 0;
}

int orc_assemble_dense(int l, const double* kappa, double* A)
{
    if (l < 1 || l > 6) return ORC_EINVAL;
    int n = 1 << l, ne = 2 * n * n, M = (n - 1) * (n - 1);
    memset(A, 0, sizeof(double) * (size_t)M * M);
    for (int e = 0; e < ne; ++e) {
        int gu[3];
        double Kl[3][3];
        orc_local_stiffness(n, e, kappa[e], gu, Kl);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (gu[a] >= 0 && gu[b] >= 0) A[(size_t)gu[a] * M + gu[b]] += Kl[a][b];
    }
    return 0;
}

int orc_load(int l, const double* f_nodal, double* b)
{
    if (l < 1 || l > 12) return ORC_EINVAL;
    int n = 1 << l, M = (n - 1) * (n - 1);
    double h = 1.0 / n;
    if (f_nodal) {
        for (int u = 0; u < M; ++u) b[u] = h * h * f_nodal[u];
        return 0;
    }
    /* f == 1: each triangle adds |T|/3 to each of its vertices (exact). */
    memset(b, 0, sizeof(double) * M);
    int ne = 2 * n * n;
    for (int e = 0; e < ne; ++e) {
        int vi[3], vj[3];
        orc_tri_nodes(n, e, vi, vj);
        for (int a = 0; a < 3; ++a) {
            int u = orc_unknown(n, vi[a], vj[a]);
            if (u >= 0) b[u] += 0.5 * h * h / 3.0;
        }
    }
    return 0;
}

/* In-place banded Cholesky A = L L^T (lower band, half-bandwidth bw) and the
 * two triangular solves. */
static int orc_band_cholesky(int M, int bw, double* band)
{
    for (int j = 0; j < M; ++j) {
        double s = band[(size_t)j * (bw + 1)];
        int k0 = j - bw > 0 ? j - bw : 0;
        for (int k = k0; k < j; ++k) {
            double v = band[(size_t)j * (bw + 1) + (j - k)];
            s -= v * v;
        }
        if (!(s > 0)) return ORC_ESING;
        double d = sqrt(s);
        band[(size_t)j * (bw + 1)] = d;
        int imax = j + bw < M - 1 ? j + bw : M - 1;
        for (int i = j + 1; i <= imax; ++i) {
            double t = band[(size_t)i * (bw + 1) + (i - j)];
            int kk0 = i - bw > 0 ? i - bw : 0;
            for (int k = kk0; k < j; ++k)
                t -= band[(size_t)i * (bw + 1) + (i - k)] * band[(size_t)j * (bw + 1) + (j - k)];
            band[(size_t)i * (bw + 1) + (i - j)] = t / d;
        }
    }
    return 0;
}

static void orc_band_solve(int M, int bw, const double* L, const double* b, double* x)
{
    for (int i = 0; i < M; ++i) {
        double s = b[i];
        int k0 = i - bw > 0 ? i - bw : 0;
        for (int k = k0; k < i; ++k) s -= L[(size_t)i * (bw + 1) + (i - k)] * x[k];
        x[i] = s / L[(size_t)i * (bw + 1)];
    }
    for (int i = M - 1; i >= 0; --i) {
        double s = x[i];
        int kmax = i + bw < M - 1 ? i + bw : M - 1;
        for (int k = i + 1; k <= kmax; ++k) s -= L[(size_t)k * (bw + 1) + (k - i)] * x[k];
        x[i] = s / L[(size_t)i * (bw + 1)];
    }
}

int orc_solve(int l, const double* kappa, const double* b, double* p)
{
    if (l < 1 || l > 12) return ORC_EINVAL;
    int n = 1 << l, M = (n - 1) * (n - 1), bw = n;
    double* band = (double*)malloc(sizeof(double) * (size_t)M * (bw + 1));
    if (!band) return ORC_ENOMEM;
    int rc = orc_assemble_band(l, kappa, band);
    if (rc == 0) rc = orc_band_cholesky(M, bw, band);
    if (rc == 0) orc_band_solve(M, bw, band, b, p);
    free(band);
    return rc;
}

/* ======================================================================
 * Observation operator (Sec. 5): p -> (p(d_o))_o, P1 interpolation.
 * ==================================================================== */
static double orc_nodal(int n, const double* p, int i, int j)
{
    int u = orc_unknown(n, i, j);
    return u < 0 ? 0.0 : p[u];
}

int orc_observe(int l, int m, const double* p, double* G)
{
    if (l < 1 || l > 12 || m < 1) return ORC_EINVAL;
    int n = 1 << l;
    for (int b = 1; b <= m; ++b)
        for (int a = 1; a <= m; ++a) {
            double x = (double)a / (double)(m + 1), y = (double)b / (double)(m + 1);
            int i = (int)floor(x * n), j = (int)floor(y * n);
            if (i > n - 1) i = n - 1;
            if (j > n - 1) j = n - 1;
            double xi = x * n - i, eta = y * n - j;
            double v;
            if (xi >= eta)
                v = (1.0 - xi) * orc_nodal(n, p, i, j) + (xi - eta) * orc_nodal(n, p, i + 1, j)
                  + eta * orc_nodal(n, p, i + 1, j + 1);
            else
                v = (1.0 - eta) * orc_nodal(n, p, i, j) + xi * orc_nodal(n, p, i + 1, j + 1)
                  + (eta - xi) * orc_nodal(n, p, i, j + 1);
            G[(b - 1) * m + (a - 1)] = v;
        }
    return 0;
}

/* potential Phi = 1/2 |Gamma^{-1/2}(y - G)|^2, Gamma = sigma_n^2 I (Sec. 2.1) */
double orc_potential(int nobs, const double* G, const double* y, double sigma_n)
{
    double s = 0.0;
    for (int o = 0; o < nobs; ++o) {
        double r = (y[o] - G[o]) / sigma_n;
        s += r * r;
    }
    return 0.5 * s;
}

int orc_forward_kappa(int l, int m, int64_t N, const double* kappa, double* G, double* p_out,
                      int nthreads)
{
    if (l < 1 || l > 12 || m < 1 || N < 0) return ORC_EINVAL;
    int n = 1 << l, ne = 2 * n * n, M = (n - 1) * (n - 1);
    int err = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(min : err)
#endif
    for (int64_t q = 0; q < N; ++q) {
        double* b = (double*)malloc(sizeof(double) * M);
        double* p = (double*)malloc(sizeof(double) * M);
        int rc = (!b || !p) ? ORC_ENOMEM : orc_load(l, NULL, b);
        if (rc == 0) rc = orc_solve(l, kappa + q * ne, b, p);
        if (rc == 0) rc = orc_observe(l, m, p, G + q * m * m);
        if (rc == 0 && p_out) memcpy(p_out + q * M, p, sizeof(double) * M);
        if (rc < err) err = rc;
        free(b); free(p);
    }
    (void)nthreads;
    return err;
}

/* ======================================================================
 * Flow cell (Sec. 5, Example 5.3): Dirichlet p = 0 / p = 1 on the left /
 * right edge, natural (no-flow) conditions on the bottom and top edges.
 * The same generic per-triangle assembly; the unknowns are the nodes off
 * the two Dirichlet edges, bottom and top rows included.
 * ==================================================================== */
static int orc_flow_unknown(int n, int i, int j)
{
    if (i < 1 || i > n - 1 || j < 0 || j > n) return -1;
    return j * (n - 1) + (i - 1);
}

/* nodal values (n+1)^2 (node j (n+1) + i) of one coefficient field */
static int orc_flow_solve_nodes(int l, const double* kappa, double* pn)
{
    int n = 1 << l, ne = 2 * n * n, M = (n - 1) * (n + 1), bw = n;
    double h = 1.0 / n;
    double* band = (double*)calloc((size_t)M * (bw + 1), sizeof(double));
    double* b = (double*)calloc((size_t)M, sizeof(double));
    double* x = (double*)malloc(sizeof(double) * (size_t)M);
    if (!band || !b || !x) { free(band); free(b); free(x); return ORC_ENOMEM; }
    int rc = 0;
    for (int e = 0; e < ne && rc == 0; ++e) {
        int vi[3], vj[3], gu[3];
        double xx[3], yy[3], g[3];
        orc_tri_nodes(n, e, vi, vj);
        for (int a = 0; a < 3; ++a) {
            xx[a] = vi[a] * h;
            yy[a] = vj[a] * h;
            gu[a] = orc_flow_unknown(n, vi[a], vj[a]);
            g[a] = vi[a] == n ? 1.0 : 0.0; /* Dirichlet value where gu < 0 */
        }
        double det = (xx[1] - xx[0]) * (yy[2] - yy[0]) - (xx[2] - xx[0]) * (yy[1] - yy[0]);
        double area = 0.5 * fabs(det), gx[3], gy[3];
        for (int a = 0; a < 3; ++a) {
            int bb = (a + 1) % 3, c = (a + 2) % 3;
            gx[a] = (yy[bb] - yy[c]) / det;
            gy[a] = (xx[c] - xx[bb]) / det;
        }
        for (int a = 0; a < 3; ++a) {
            if (gu[a] < 0) continue;
            for (int bb = 0; bb < 3; ++bb) {
                double kab = kappa[e] * area * (gx[a] * gx[bb] + gy[a] * gy[bb]);
                if (gu[bb] < 0) {
                    b[gu[a]] -= kab * g[bb]; /* lift the known value */
                    continue;
                }
                if (gu[bb] > gu[a]) continue;
                int k = gu[a] - gu[bb];
                if (k > bw) { rc = ORC_EINVAL; break; }
                band[(size_t)gu[a] * (bw + 1) + k] += kab;
            }
        }
    }
    if (rc == 0) rc = orc_band_cholesky(M, bw, band);
    if (rc == 0) {
        orc_band_solve(M, bw, band, b, x);
        for (int j = 0; j <= n; ++j)
            for (int i = 0; i <= n; ++i) {
                int u = orc_flow_unknown(n, i, j);
                pn[j * (n + 1) + i] = u >= 0 ? x[u] : (i == n ? 1.0 : 0.0);
            }
    }
    free(band); free(b); free(x);
    return rc;
}

int orc_flow_forward_kappa(int l, int m, int64_t N, const double* kappa, double* G, double* p_out,
                           int nthreads)
{
    if (l < 1 || l > 12 || m < 1 || N < 0) return ORC_EINVAL;
    int n = 1 << l, ne = 2 * n * n, M = (n - 1) * (n + 1);
    int err = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(min : err)
#endif
    for (int64_t q = 0; q < N; ++q) {
        double* pn = (double*)malloc(sizeof(double) * (size_t)(n + 1) * (n + 1));
        int rc = pn ? orc_flow_solve_nodes(l, kappa + q * ne, pn) : ORC_ENOMEM;
        if (rc == 0) {
            for (int bb = 1; bb <= m; ++bb)
                for (int a = 1; a <= m; ++a) {
                    double x = (double)a / (double)(m + 1), y = (double)bb / (double)(m + 1);
                    int i = (int)floor(x * n), j = (int)floor(y * n);
                    if (i > n - 1) i = n - 1;
                    if (j > n - 1) j = n - 1;
                    double xi = x * n - i, eta = y * n - j;
                    const double* P = pn;
                    int s = n + 1;
                    double v;
                    if (xi >= eta)
                        v = (1.0 - xi) * P[j * s + i] + (xi - eta) * P[j * s + i + 1] + eta * P[(j + 1) * s + i + 1];
                    else
                        v = (1.0 - eta) * P[j * s + i] + xi * P[(j + 1) * s + i + 1] + (eta - xi) * P[(j + 1) * s + i];
                    G[q * m * m + (bb - 1) * m + (a - 1)] = v;
                }
            if (p_out)
                for (int j = 0; j <= n; ++j)
                    for (int i = 1; i <= n - 1; ++i) p_out[q * M + orc_flow_unknown(n, i, j)] = pn[j * (n + 1) + i];
        }
        if (rc < err) err = rc;
        free(pn);
    }
    (void)nthreads;
    return err;
}

int orc_forward(int l, int K, double sigma2, double corr_len, int m, int64_t N,
                const double* theta, double* G, int nthreads)
{
    if (l < 1 || l > 12 || K <= 0 || N < 0) return ORC_EINVAL;
    int n = 1 << l, ne = 2 * n * n;
    double* B = (double*)malloc(sizeof(double) * (size_t)K * ne);
    double* kappa = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * ne);
    if (!B || !kappa) { free(B); free(kappa); return ORC_ENOMEM; }
    int rc = orc_kl_basis(l, K, sigma2, corr_len, B);
    if (rc == 0) {
        orc_kl_field(l, K, N, B, theta, kappa);
        for (int64_t i = 0; i < N * ne; ++i) kappa[i] = exp(kappa[i]);
        rc = orc_forward_kappa(l, m, N, kappa, G, NULL, nthreads);
    }
    free(B); free(kappa);
    return rc;
}

/* ======================================================================
 * Adaptive step (Sec. 3.4).  Incremental log-weights lw_j(t) = -t*scale*d_j
 * (tempering, Sec. 3.1: d = Phi, scale = 1; bridging, Sec. 3.2/4.1:
 * d = Phi_{l+1} - Phi_l, scale = beta).  ESS = J/(1+cv^2) with the
 * population variance, which equals (sum w)^2 / sum w^2.
 * ==================================================================== */
double orc_ess(int64_t N, const double* d, double scale, double t)
{
    double mx = -INFINITY;
    for (int64_t j = 0; j < N; ++j) {
        double lw = -t * scale * d[j];
        if (lw > mx) mx = lw;
    }
    double s1 = 0.0, s2 = 0.0;
    for (int64_t j = 0; j < N; ++j) {
        double v = exp(-t * scale * d[j] - mx);
        s1 += v; s2 += v * v;
    }
    return s1 * s1 / s2;
}

/* The argmin of (ESS(cur+t) - tau)^2 over t in [min(eps,1-cur), 1-cur].
 * ESS is non-increasing in t, so the minimiser is the right end if it still
 * meets the target, the left end if even that misses it, and otherwise the
 * root, located by 64 bisection steps that keep ESS(lo) >= tau > ESS(hi).  */
int orc_next_step(int64_t N, const double* d, double scale, double cur, double tau_ess,
                  double eps, double* next, double* logw, double* w, double* dlogZ, double* ess)
{
    if (N <= 0 || !(cur >= 0.0 && cur < 1.0) || !(eps > 0)) return ORC_EINVAL;
    for (int64_t j = 0; j < N; ++j)
        if (!isfinite(d[j])) return ORC_EINVAL;
    double tmax = 1.0 - cur;
    double tmin = eps < tmax ? eps : tmax;
    double t;
    int at_end = 0;
    if (orc_ess(N, d, scale, tmax) >= tau_ess) { t = tmax; at_end = 1; }
    else if (orc_ess(N, d, scale, tmin) <= tau_ess) { t = tmin; at_end = (tmin == tmax); }
    else {
        double lo = tmin, hi = tmax;
        for (int it = 0; it < 64; ++it) {
            double mid = 0.5 * (lo + hi);
            if (orc_ess(N, d, scale, mid) >= tau_ess) lo = mid; else hi = mid;
        }
        t = lo;
    }
    *next = at_end ? 1.0 : cur + t;
    /* weights at the chosen t, log-sum-exp normalised (Sec. 2.3) */
    double mx = -INFINITY;
    for (int64_t j = 0; j < N; ++j) {
        logw[j] = -t * scale * d[j];
        if (logw[j] > mx) mx = logw[j];
    }
    double s = 0.0;
    for (int64_t j = 0; j < N; ++j) s += exp(logw[j] - mx);
    double lse = mx + log(s);
    for (int64_t j = 0; j < N; ++j) w[j] = exp(logw[j] - lse);
    *dlogZ = lse - log((double)N);
    *ess = orc_ess(N, d, scale, t);
    return 0;
}

/* ======================================================================
 * Multinomial resampling (Sec. 2.4) by an exact integer CDF.  Weights are
 * scaled by the power of two that brings the largest into [1/2,1), then
 * quantised to q_j = floor(w_j 2^(62-c)), c = ceil(log2 N); every step is
 * exact, so the ancestors depend only on (w, u).
 * ==================================================================== */
static int orc_ceil_log2(int64_t N)
{
    int c = 0;
    while (((int64_t)1 << c) < N) ++c;
    return c;
}

int orc_resample(int64_t N, const double* w, const double* u, int32_t* anc)
{
    if (N <= 0 || N > (1 << 30)) return ORC_EINVAL;
    double mx = 0.0;
    for (int64_t j = 0; j < N; ++j) {
        if (!(w[j] >= 0.0) || isinf(w[j])) return ORC_EINVAL;
        if (w[j] > mx) mx = w[j];
    }
    if (!(mx > 0.0)) return ORC_ESING;
    int ex;
    frexp(mx, &ex); /* mx = f 2^ex, f in [1/2,1) */
    int c = orc_ceil_log2(N);
    uint64_t* C = (uint64_t*)malloc(sizeof(uint64_t) * N);
    if (!C) return ORC_ENOMEM;
    uint64_t run = 0;
    for (int64_t j = 0; j < N; ++j) {
        double v = ldexp(ldexp(w[j], -ex), 62 - c);
        run += (uint64_t)floor(v);
        C[j] = run;
    }
    uint64_t T = run;
    for (int64_t i = 0; i < N; ++i) {
        if (!(u[i] >= 0.0 && u[i] < 1.0)) { free(C); return ORC_EINVAL; }
        uint64_t U = (uint64_t)ldexp(u[i], 53);
        unsigned __int128 prod = (unsigned __int128)U * T;
        uint64_t ti = (uint64_t)(prod >> 53);
        int64_t lo = 0, hi = N - 1; /* smallest j with C[j] > ti */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (C[mid] > ti) hi = mid; else lo = mid + 1;
        }
        anc[i] = (int32_t)lo;
    }
    free(C);
    return 0;
}

/* ======================================================================
 * pCN proposal (Cotter, Roberts, Stuart, White; cited in Sec. 1 and
 * Sec. 5) for a N(0, I) prior: theta' = sqrt(1-s^2) theta + s xi.  It is
 * reversible w.r.t. the prior, so the Metropolis-Hastings ratio contains
 * only the potential of the current target.
 * ==================================================================== */
void orc_pcn_propose(int64_t N, int K, double s, const double* theta, const double* xi,
                     double* theta_new)
{
    double a = sqrt(1.0 - s * s);
    for (int64_t i = 0; i < N * K; ++i) theta_new[i] = a * theta[i] + s * xi[i];
}

void orc_rwm_propose(int64_t N, int K, double s, const double* theta, const double* xi,
                     double* theta_new)
{
    for (int64_t i = 0; i < N * K; ++i) theta_new[i] = theta[i] + s * xi[i];
}

int orc_mh_accept(double psi_old, double psi_new, double u)
{
    return log(u) < -(psi_new - psi_old);
}

int orc_da_accept(double psi_old, double psi_new, double psis_old, double psis_new, double u1,
                  double u2, int* stage1)
{
    int s1 = log(u1) < -(psis_new - psis_old);
    if (stage1) *stage1 = s1;
    if (!s1) return 0;
    return log(u2) < -(psi_new - psi_old) + (psis_new - psis_old);
}

/* ======================================================================
 * The MLS^2MC sampler (Sec. 4), update scheme of Sec. 4.4: the first update
 * and every update after a level update are tempering updates; otherwise
 * cv^LU is estimated on the first J_tilde particles and a level update is
 * taken when cv^LU >= tau_LU.  At beta = 1 the remaining levels are bridged.
 * Random streams: 0 prior, 3 resampling, 4 pCN normals, 5 pCN uniforms.
 * ==================================================================== */
enum { ST_PRIOR = 0, ST_RESAMPLE = 3, ST_PCN_XI = 4, ST_PCN_U = 5, ST_PCN_U2 = 6 };

typedef struct {
    const orc_config* cfg;
    int nobs;
    double* B[16]; /* KL bases per level (PDE model) */
} orc_model;

static int orc_model_eval(orc_model* md, int l, int64_t N, const double* theta, double* G)
{
    const orc_config* cfg = md->cfg;
    int K = cfg->K;
    if (cfg->model == ORC_MODEL_LINEAR) {
        double sc = ldexp(1.0, -2 * l);
        for (int64_t q = 0; q < N; ++q)
            for (int o = 0; o < md->nobs; ++o) {
                double s = 0.0;
                for (int k = 0; k < K; ++k)
                    s += (cfg->lin_A[o * K + k] + sc * cfg->lin_E[o * K + k]) * theta[q * K + k];
                G[q * md->nobs + o] = s;
            }
        return 0;
    }
    int n = 1 << l, ne = 2 * n * n;
    if (!md->B[l]) {
        md->B[l] = (double*)malloc(sizeof(double) * (size_t)K * ne);
        if (!md->B[l]) return ORC_ENOMEM;
        int rc = orc_kl_basis(l, K, cfg->sigma2, cfg->corr_len, md->B[l]);
        if (rc) return rc;
    }
    double* kap = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * ne);
    if (!kap) return ORC_ENOMEM;
    orc_kl_field(l, K, N, md->B[l], theta, kap);
    for (int64_t i = 0; i < N * ne; ++i) kap[i] = exp(kap[i]);
    int rc = cfg->model == ORC_MODEL_FLOWCELL ? orc_flow_forward_kappa(l, cfg->m, N, kap, G, NULL, cfg->nthreads)
                                              : orc_forward_kappa(l, cfg->m, N, kap, G, NULL, cfg->nthreads);
    free(kap);
    return rc;
}

static void orc_potentials(orc_model* md, int64_t N, const double* G, const double* y, double* phi)
{
    for (int64_t q = 0; q < N; ++q) phi[q] = orc_potential(md->nobs, G + q * md->nobs, y, md->cfg->sigma_n);
}

typedef struct {
    double *theta, *Glo, *Ghi, *philo, *phihi;
} orc_state;

static void orc_gather(int64_t J, int K, int nobs, const int32_t* anc, orc_state* s, orc_state* tmp,
                       int with_hi)
{
    for (int64_t i = 0; i < J; ++i) {
        int64_t a = anc[i];
        memcpy(tmp->theta + i * K, s->theta + a * K, sizeof(double) * K);
        memcpy(tmp->Glo + i * nobs, s->Glo + a * nobs, sizeof(double) * nobs);
        tmp->philo[i] = s->philo[a];
        if (with_hi) {
            memcpy(tmp->Ghi + i * nobs, s->Ghi + a * nobs, sizeof(double) * nobs);
            tmp->phihi[i] = s->phihi[a];
        }
    }
    memcpy(s->theta, tmp->theta, sizeof(double) * J * K);
    memcpy(s->Glo, tmp->Glo, sizeof(double) * J * nobs);
    memcpy(s->philo, tmp->philo, sizeof(double) * J);
    if (with_hi) {
        memcpy(s->Ghi, tmp->Ghi, sizeof(double) * J * nobs);
        memcpy(s->phihi, tmp->phihi, sizeof(double) * J);
    }
}

/* n_mcmc pCN steps targeting exp(-beta[(1-zeta)Phi_lo + zeta Phi_hi]) times
 * the prior.  bridge = 0: only Phi_lo (level l) is used (zeta ignored).    */
/* surrogate potential beta * Phi(S theta) of the delayed-acceptance stage 1 */
static double orc_sur_psi(const orc_config* cfg, int nobs, const double* th, const double* y,
                          double beta)
{
    double ph = 0.0;
    for (int o = 0; o < nobs; ++o) {
        double g = 0.0;
        for (int k = 0; k < cfg->K; ++k) g += cfg->da_S[o * cfg->K + k] * th[k];
        double r = (y[o] - g) / cfg->sigma_n;
        ph += r * r;
    }
    return beta * 0.5 * ph;
}

static int orc_mutate(orc_model* md, const double* y, int stage, int l, int bridge, double beta,
                      double zeta, double s_pcn, orc_state* s, int64_t* solves, int64_t* acc,
                      int64_t* prop, int64_t* pass1)
{
    const orc_config* cfg = md->cfg;
    int64_t J = cfg->J;
    int K = cfg->K, nobs = md->nobs;
    int need_lo = !bridge || zeta < 1.0;
    int need_hi = bridge;
    double* xi = (double*)malloc(sizeof(double) * J * K);
    double* th = (double*)malloc(sizeof(double) * J * K);
    double* Gl = (double*)malloc(sizeof(double) * J * nobs);
    double* Gh = (double*)malloc(sizeof(double) * J * nobs);
    double* pl = (double*)malloc(sizeof(double) * J);
    double* ph = (double*)malloc(sizeof(double) * J);
    int rc = (!xi || !th || !Gl || !Gh || !pl || !ph) ? ORC_ENOMEM : 0;
    for (int mstep = 0; rc == 0 && mstep < cfg->n_mcmc; ++mstep) {
        for (int64_t i = 0; i < J * K; ++i)
            xi[i] = orc_normal(cfg->seed, ST_PCN_XI, (uint32_t)stage, (uint32_t)mstep, (uint32_t)i);
        if (cfg->kernel == 1) orc_rwm_propose(J, K, s_pcn, s->theta, xi, th);
        else orc_pcn_propose(J, K, s_pcn, s->theta, xi, th);
        if (need_lo) {
            rc = orc_model_eval(md, l, J, th, Gl);
            if (rc) break;
            orc_potentials(md, J, Gl, y, pl);
            solves[l] += J;
        }
        if (need_hi) {
            rc = orc_model_eval(md, l + 1, J, th, Gh);
            if (rc) break;
            orc_potentials(md, J, Gh, y, ph);
            solves[l + 1] += J;
        }
        for (int64_t j = 0; j < J; ++j) {
            double psi_old, psi_new;
            if (!bridge) { psi_old = beta * s->philo[j]; psi_new = beta * pl[j]; }
            else if (zeta < 1.0) {
                psi_old = beta * ((1.0 - zeta) * s->philo[j] + zeta * s->phihi[j]);
                psi_new = beta * ((1.0 - zeta) * pl[j] + zeta * ph[j]);
            } else { psi_old = beta * s->phihi[j]; psi_new = beta * ph[j]; }
            if (cfg->kernel == 1) {  /* random walk: the N(0, I) prior does not cancel */
                double qo = 0.0, qn = 0.0;
                for (int k = 0; k < K; ++k) {
                    qo += s->theta[j * K + k] * s->theta[j * K + k];
                    qn += th[j * K + k] * th[j * K + k];
                }
                psi_old += 0.5 * qo;
                psi_new += 0.5 * qn;
            }
            double u = orc_uniform(cfg->seed, ST_PCN_U, (uint32_t)stage, (uint32_t)mstep, (uint32_t)j);
            ++*prop;
            int ok;
            if (cfg->da_S) {
                double u2 = orc_uniform(cfg->seed, ST_PCN_U2, (uint32_t)stage, (uint32_t)mstep, (uint32_t)j);
                int s1;
                ok = orc_da_accept(psi_old, psi_new, orc_sur_psi(cfg, nobs, s->theta + j * K, y, beta),
                                   orc_sur_psi(cfg, nobs, th + j * K, y, beta), u, u2, &s1);
                *pass1 += s1;
            } else {
                ok = orc_mh_accept(psi_old, psi_new, u);
            }
            if (ok) {
                ++*acc;
                memcpy(s->theta + j * K, th + j * K, sizeof(double) * K);
                if (need_lo) { memcpy(s->Glo + j * nobs, Gl + j * nobs, sizeof(double) * nobs); s->philo[j] = pl[j]; }
                if (need_hi) { memcpy(s->Ghi + j * nobs, Gh + j * nobs, sizeof(double) * nobs); s->phihi[j] = ph[j]; }
            }
        }
    }
    free(xi); free(th); free(Gl); free(Gh); free(pl); free(ph);
    return rc;
}

/* pCN step adaptation towards an acceptance rate of 1/4 (an extension) */
static double orc_adapt_step(double s, int64_t acc, int64_t prop)
{
    double a = prop > 0 ? (double)acc / (double)prop : 0.25;
    double t = s * exp(2.0 * (a - 0.25));
    return t < 0.005 ? 0.005 : (t > 1.0 ? 1.0 : t);
}

static void orc_log_stage(orc_result* r, int type, int level, double beta, double zeta, double ess,
                          double step, double acc_rate)
{
    int s = r->n_stages;
    if (s < r->max_stage_log) {
        if (r->stage_step) r->stage_step[s] = step;
        if (r->stage_acc_rate) r->stage_acc_rate[s] = acc_rate;
        if (r->stage_type) r->stage_type[s] = type;
        if (r->stage_level) r->stage_level[s] = level;
        if (r->stage_beta) r->stage_beta[s] = beta;
        if (r->stage_zeta) r->stage_zeta[s] = zeta;
        if (r->stage_ess) r->stage_ess[s] = ess;
    }
    r->n_stages = s + 1;
}

int orc_run_sampler(const orc_config* cfg, const double* y, double* theta_out, orc_result* res)
{
    if (!cfg || !y || !res || cfg->J <= 0 || cfg->K <= 0 || cfg->l_min < 0 || cfg->l_max < cfg->l_min
        || cfg->l_max > 12 || cfg->n_mcmc < 0 || cfg->J_tilde < 1 || cfg->J_tilde > cfg->J)
        return ORC_EINVAL;
    if (cfg->model != ORC_MODEL_LINEAR && cfg->l_min < 1) return ORC_EINVAL;
    orc_model md;
    memset(&md, 0, sizeof(md));
    md.cfg = cfg;
    md.nobs = cfg->model == ORC_MODEL_LINEAR ? cfg->nobs : cfg->m * cfg->m;
    int64_t J = cfg->J, Jt = cfg->J_tilde;
    int K = cfg->K, nobs = md.nobs;
    res->n_stages = 0; res->log_Z = 0.0;
    memset(res->solves, 0, sizeof(res->solves));
    res->accepted = res->proposed = 0;
    res->stage1_passed = 0;
    if (cfg->da_S && cfg->model != ORC_MODEL_LINEAR) return ORC_EINVAL;

    orc_state s, tmp;
    double* buf = (double*)malloc(sizeof(double) * 2 * (J * K + 2 * J * nobs + 2 * J));
    double* d = (double*)malloc(sizeof(double) * J);
    double* lw = (double*)malloc(sizeof(double) * J);
    double* w = (double*)malloc(sizeof(double) * J);
    double* u = (double*)malloc(sizeof(double) * J);
    int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * J);
    if (!buf || !d || !lw || !w || !u || !anc) {
        free(buf); free(d); free(lw); free(w); free(u); free(anc);
        return ORC_ENOMEM;
    }
    double* p = buf;
    s.theta = p; p += J * K; s.Glo = p; p += J * nobs; s.Ghi = p; p += J * nobs;
    s.philo = p; p += J; s.phihi = p; p += J;
    tmp.theta = p; p += J * K; tmp.Glo = p; p += J * nobs; tmp.Ghi = p; p += J * nobs;
    tmp.philo = p; p += J; tmp.phihi = p; p += J;

    int rc = 0;
    /* prior draw (Sec. 2.4: independent samples of nu_0 = mu_0) */
    for (int64_t i = 0; i < J * K; ++i) s.theta[i] = orc_normal(cfg->seed, ST_PRIOR, 0, 0, (uint32_t)i);
    int l = cfg->l_min;
    double beta = 0.0;
    double s_pcn = cfg->s_pcn;
    int prev_lu = 1; /* u(-1) = (0,0): the first update is a tempering update */
    rc = orc_model_eval(&md, l, J, s.theta, s.Glo);
    if (rc == 0) { orc_potentials(&md, J, s.Glo, y, s.philo); res->solves[l] += J; }
    int stage = 0;
    while (rc == 0) {
        if (beta == 1.0 && l == cfg->l_max) break;
        if (stage >= cfg->max_stages) { rc = ORC_ESING; break; }
        int do_lu, checked = 0;
        double cv = 0.0;
        /* look-ahead: cv^LU of a level update at the current beta, from the
         * first J_tilde particles (Sec. 4.4) */
#define ORC_LOOK_AHEAD()                                                                  \
        do {                                                                              \
            rc = orc_model_eval(&md, l + 1, Jt, s.theta, s.Ghi);                          \
            if (rc) break;                                                                \
            orc_potentials(&md, Jt, s.Ghi, y, s.phihi);                                   \
            res->solves[l + 1] += Jt;                                                     \
            for (int64_t j = 0; j < Jt; ++j) d[j] = s.phihi[j] - s.philo[j];             \
            double ess_ = orc_ess(Jt, d, beta, 1.0);                                      \
            cv = sqrt((double)Jt / ess_ - 1.0 > 0 ? (double)Jt / ess_ - 1.0 : 0.0);       \
            checked = 1;                                                                  \
        } while (0)
        if (beta == 1.0) {
            if (cfg->tau_min > 0.0) {  /* scheme u' (Sec. 4.5) */
                ORC_LOOK_AHEAD();
                if (rc) break;
                if (cv < cfg->tau_min) break;  /* terminate on level l */
            }
            do_lu = 1;
        } else if (cfg->scheme == 1 || l == cfg->l_max || prev_lu) {
            do_lu = 0;
        } else {
            ORC_LOOK_AHEAD();
            if (rc) break;
            do_lu = !(cv < cfg->tau_lu);
        }
#undef ORC_LOOK_AHEAD
        if (!do_lu) {
            /* tempering update (Sec. 3.1) */
            double nb, dlz, ess;
            rc = orc_next_step(J, s.philo, 1.0, beta, cfg->tau_ess, cfg->eps, &nb, lw, w, &dlz, &ess);
            if (rc) break;
            res->log_Z += dlz;
            for (int64_t i = 0; i < J; ++i) u[i] = orc_uniform(cfg->seed, ST_RESAMPLE, (uint32_t)stage, 0, (uint32_t)i);
            rc = orc_resample(J, w, u, anc);
            if (rc) break;
            orc_gather(J, K, nobs, anc, &s, &tmp, 0);
            const int64_t a0 = res->accepted;
            const double s_used = s_pcn;
            rc = orc_mutate(&md, y, stage, l, 0, nb, 1.0, s_pcn, &s, res->solves, &res->accepted,
                            &res->proposed, &res->stage1_passed);
            if (rc) break;
            if (cfg->s_adapt) s_pcn = orc_adapt_step(s_pcn, res->accepted - a0, J * cfg->n_mcmc);
            beta = nb;
            orc_log_stage(res, checked ? 1 : 0, l, beta, 0.0, ess, s_used,
                          cfg->n_mcmc ? (double)(res->accepted - a0) / (double)(J * cfg->n_mcmc) : 0.0);
            ++stage;
            prev_lu = 0;
        } else {
            /* level update: bridge Phi_l -> Phi_{l+1} at inverse temperature beta */
            int64_t j0 = checked ? Jt : 0;
            if (J - j0 > 0) {
                rc = orc_model_eval(&md, l + 1, J - j0, s.theta + j0 * K, s.Ghi + j0 * nobs);
                if (rc) break;
                orc_potentials(&md, J - j0, s.Ghi + j0 * nobs, y, s.phihi + j0);
                res->solves[l + 1] += J - j0;
            }
            double zeta = 0.0;
            int first = 1;
            while (zeta < 1.0) {
                if (stage >= cfg->max_stages) { rc = ORC_ESING; break; }
                for (int64_t j = 0; j < J; ++j) d[j] = s.phihi[j] - s.philo[j];
                double nz, dlz, ess;
                rc = orc_next_step(J, d, beta, zeta, cfg->tau_ess, cfg->eps, &nz, lw, w, &dlz, &ess);
                if (rc) break;
                res->log_Z += dlz;
                for (int64_t i = 0; i < J; ++i) u[i] = orc_uniform(cfg->seed, ST_RESAMPLE, (uint32_t)stage, 0, (uint32_t)i);
                rc = orc_resample(J, w, u, anc);
                if (rc) break;
                orc_gather(J, K, nobs, anc, &s, &tmp, 1);
                const int64_t a0 = res->accepted;
                const double s_used = s_pcn;
                rc = orc_mutate(&md, y, stage, l, 1, beta, nz, s_pcn, &s, res->solves, &res->accepted,
                                &res->proposed, &res->stage1_passed);
                if (rc) break;
                if (cfg->s_adapt) s_pcn = orc_adapt_step(s_pcn, res->accepted - a0, J * cfg->n_mcmc);
                zeta = nz;
                orc_log_stage(res, first ? (checked ? 2 : 3) : 4, l + 1, beta, zeta, ess, s_used,
                              cfg->n_mcmc ? (double)(res->accepted - a0) / (double)(J * cfg->n_mcmc) : 0.0);
                first = 0;
                ++stage;
            }
            if (rc) break;
            ++l;
            memcpy(s.Glo, s.Ghi, sizeof(double) * J * nobs);
            memcpy(s.philo, s.phihi, sizeof(double) * J);
            prev_lu = 1;
        }
    }
    res->final_level = l;
    res->final_beta = beta;
    if (rc == 0) memcpy(theta_out, s.theta, sizeof(double) * J * K);
    for (int i = 0; i < 16; ++i) free(md.B[i]);
    free(buf); free(d); free(lw); free(w); free(u); free(anc);
    return rc;
}

/* ======================================================================
 * MLP reference: x -> GELU(W1 x + b1) -> GELU(W2 . + b2) -> W3 . + b3,
 * GELU(z) = z Phi(z) = z (1 + erf(z/sqrt 2))/2.  Loss = mean of (out-t)^2/2
 * over batch and outputs.
 * ==================================================================== */
static double orc_gelu(double z) { return 0.5 * z * (1.0 + erf(z * M_SQRT1_2)); }
static double orc_gelu_d(double z)
{
    return 0.5 * (1.0 + erf(z * M_SQRT1_2)) + z * exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
}

int orc_mlp_forward(int D, int H1, int H2, int O, const double* P, int64_t B, const double* x,
                    double* out)
{
    const double *W1 = P, *b1 = W1 + (size_t)H1 * D, *W2 = b1 + H1, *b2 = W2 + (size_t)H2 * H1,
                 *W3 = b2 + H2, *b3 = W3 + (size_t)O * H2;
    double* h1 = (double*)malloc(sizeof(double) * H1);
    double* h2 = (double*)malloc(sizeof(double) * H2);
    if (!h1 || !h2) { free(h1); free(h2); return ORC_ENOMEM; }
    for (int64_t q = 0; q < B; ++q) {
        for (int i = 0; i < H1; ++i) {
            double s = b1[i];
            for (int k = 0; k < D; ++k) s += W1[(size_t)i * D + k] * x[q * D + k];
            h1[i] = orc_gelu(s);
        }
        for (int i = 0; i < H2; ++i) {
            double s = b2[i];
            for (int k = 0; k < H1; ++k) s += W2[(size_t)i * H1 + k] * h1[k];
            h2[i] = orc_gelu(s);
        }
        for (int i = 0; i < O; ++i) {
            double s = b3[i];
            for (int k = 0; k < H2; ++k) s += W3[(size_t)i * H2 + k] * h2[k];
            out[q * O + i] = s;
        }
    }
    free(h1); free(h2);
    return 0;
}

int orc_mlp_loss_grad(int D, int H1, int H2, int O, const double* P, int64_t B, const double* x,
                      const double* target, double* loss, double* grad)
{
    const double *W1 = P, *b1 = W1 + (size_t)H1 * D, *W2 = b1 + H1, *b2 = W2 + (size_t)H2 * H1,
                 *W3 = b2 + H2, *b3 = W3 + (size_t)O * H2;
    size_t np = (size_t)H1 * D + H1 + (size_t)H2 * H1 + H2 + (size_t)O * H2 + O;
    double *gW1 = grad, *gb1 = gW1 + (size_t)H1 * D, *gW2 = gb1 + H1, *gb2 = gW2 + (size_t)H2 * H1,
           *gW3 = gb2 + H2, *gb3 = gW3 + (size_t)O * H2;
    memset(grad, 0, sizeof(double) * np);
    double* z1 = (double*)malloc(sizeof(double) * H1);
    double* h1 = (double*)malloc(sizeof(double) * H1);
    double* z2 = (double*)malloc(sizeof(double) * H2);
    double* h2 = (double*)malloc(sizeof(double) * H2);
    double* g3 = (double*)malloc(sizeof(double) * O);
    double* g2 = (double*)malloc(sizeof(double) * H2);
    double* g1 = (double*)malloc(sizeof(double) * H1);
    if (!z1 || !h1 || !z2 || !h2 || !g3 || !g2 || !g1) {
        free(z1); free(h1); free(z2); free(h2); free(g3); free(g2); free(g1);
        return ORC_ENOMEM;
    }
    double L = 0.0, scale = 1.0 / ((double)B * O);
    for (int64_t q = 0; q < B; ++q) {
        for (int i = 0; i < H1; ++i) {
            double s = b1[i];
            for (int k = 0; k < D; ++k) s += W1[(size_t)i * D + k] * x[q * D + k];
            z1[i] = s; h1[i] = orc_gelu(s);
        }
        for (int i = 0; i < H2; ++i) {
            double s = b2[i];
            for (int k = 0; k < H1; ++k) s += W2[(size_t)i * H1 + k] * h1[k];
            z2[i] = s; h2[i] = orc_gelu(s);
        }
        for (int i = 0; i < O; ++i) {
            double s = b3[i];
            for (int k = 0; k < H2; ++k) s += W3[(size_t)i * H2 + k] * h2[k];
            double r = s - target[q * O + i];
            L += 0.5 * r * r;
            g3[i] = r * scale;
        }
        for (int i = 0; i < O; ++i) {
            gb3[i] += g3[i];
            for (int k = 0; k < H2; ++k) gW3[(size_t)i * H2 + k] += g3[i] * h2[k];
        }
        for (int k = 0; k < H2; ++k) {
            double s = 0.0;
            for (int i = 0; i < O; ++i) s += W3[(size_t)i * H2 + k] * g3[i];
            g2[k] = s * orc_gelu_d(z2[k]);
        }
        for (int i = 0; i < H2; ++i) {
            gb2[i] += g2[i];
            for (int k = 0; k < H1; ++k) gW2[(size_t)i * H1 + k] += g2[i] * h1[k];
        }
        for (int k = 0; k < H1; ++k) {
            double s = 0.0;
            for (int i = 0; i < H2; ++i) s += W2[(size_t)i * H1 + k] * g2[i];
            g1[k] = s * orc_gelu_d(z1[k]);
        }
        for (int i = 0; i < H1; ++i) {
            gb1[i] += g1[i];
            for (int k = 0; k < D; ++k) gW1[(size_t)i * D + k] += g1[i] * x[q * D + k];
        }
    }
    *loss = L * scale;
    free(z1); free(h1); free(z2); free(h2); free(g3); free(g2); free(g1);
    return 0;
}
