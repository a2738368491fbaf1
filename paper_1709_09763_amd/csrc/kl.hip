// Truncated Karhunen-Loeve field of the prior (Sec. 5, truncated KL
// expansion; Sec. 2.2, parameter discretisation), evaluated at the element
// centroids as a GEMM  A[N x n_e] = Theta[N x K] B_l[K x n_e]  on the CDNA4
// matrix cores.  The modes of the separable exponential covariance
// sigma2 exp(-|dx1|/c) exp(-|dx2|/c) are built here in closed form; those of
// the Matern covariance in kl_matern.hip.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "common.h"

namespace mls {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- modes --
// 1-D eigenpairs on [0,1] of exp(-|s-t|/corr): with c = 1/corr the
// eigenfunctions are (w/c) cos(wt) + sin(wt) where w solves
// (w^2 - c^2) sin w = 2 c w cos w, one root in each ((n-1) pi, n pi), and the
// eigenvalue is 2c / (w^2 + c^2).  Roots by safeguarded Newton.
static double kl_root(int n, double c)
{
    auto g = [c](double w) { return (w * w - c * c) * std::sin(w) - 2.0 * c * w * std::cos(w); };
    auto dg = [c](double w) {
        return (2.0 * w + 2.0 * c * w) * std::sin(w) + (w * w - c * c - 2.0 * c) * std::cos(w);
    };
    double lo = (n - 1) * M_PI, hi = n * M_PI;
    double glo = (n == 1) ? -1.0 : g(lo);  // g < 0 just above 0
    double w = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double gw = g(w);
        if (gw == 0.0) break;
        if ((gw < 0) == (glo < 0)) lo = w; else hi = w;
        double step = gw / dg(w);
        double wn = w - step;
        if (!(wn > lo && wn < hi)) wn = 0.5 * (lo + hi);
        if (std::fabs(wn - w) <= 4e-16 * w) { w = wn; break; }
        w = wn;
    }
    return w;
}

// Gauss-Legendre nodes/weights on [-1,1] by Newton on P_n.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wt)
{
    x.resize(n);
    wt.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                x[i] = z;
                wt[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                break;
            }
        }
    }
}

// L2(0,1) norm of (a cos wt + sin wt) by composite Gauss-Legendre.
static double l2_norm_1d(double w, double a, const std::vector<double>& gx,
                         const std::vector<double>& gw)
{
    int nsub = 4 + (int)std::ceil(w / 2.0);
    double h = 1.0 / nsub, s = 0.0;
    for (int q = 0; q < nsub; ++q)
        for (size_t i = 0; i < gx.size(); ++i) {
            double t = (q + 0.5 * (gx[i] + 1.0)) * h;
            double v = a * std::cos(w * t) + std::sin(w * t);
            s += 0.5 * h * gw[i] * v * v;
        }
    return std::sqrt(s);
}

__global__ void kl_basis_kernel(const double* __restrict__ modes, int K, int l, int64_t ne,
                                double* __restrict__ B, __hip_bfloat16* __restrict__ Bt16,
                                int Kp)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (e >= ne) return;
    const int n = 1 << l;
    const int64_t cell = e >> 1;
    const int i = (int)(cell & (n - 1)), j = (int)(cell >> l);
    double x, y;
    if ((e & 1) == 0) {
        x = (double)(3 * i + 2) / (double)(3 * n);
        y = (double)(3 * j + 1) / (double)(3 * n);
    } else {
        x = (double)(3 * i + 1) / (double)(3 * n);
        y = (double)(3 * j + 2) / (double)(3 * n);
    }
    const double* m = modes + 7 * k;  // sqrt_lam, wx, wy, ax, ay, ix, iy
    double fx = (m[3] * cos(m[1] * x) + sin(m[1] * x)) * m[5];
    double fy = (m[4] * cos(m[2] * y) + sin(m[2] * y)) * m[6];
    double v = m[0] * fx * fy;
    B[(int64_t)k * ne + e] = v;
    if (Bt16) Bt16[e * Kp + k] = __float2bfloat16((float)v);
}

int build_kl_tables(mls2mc_ctx* ctx)
{
    const mls2mc_problem& p = ctx->prob;
    if (p.cov == MLS2MC_COV_MATERN32) return build_matern_tables(ctx);
    const int K = p.K;
    const double c = 1.0 / p.corr_len;
    const int nm = K;  // 1-D modes needed at most
    std::vector<double> om(nm), mu(nm);
    for (int n = 1; n <= nm; ++n) {
        om[n - 1] = kl_root(n, c);
        mu[n - 1] = 2.0 * c / (om[n - 1] * om[n - 1] + c * c);
    }
    // first K products, descending; exact (i,j)/(j,i) ties -> smaller i first
    struct Pair { double v; int i, j; };
    std::vector<Pair> all;
    all.reserve((size_t)nm * nm);
    for (int i = 0; i < nm; ++i)
        for (int j = 0; j < nm; ++j) all.push_back({mu[i] * mu[j], i, j});
    std::partial_sort(all.begin(), all.begin() + K, all.end(), [](const Pair& a, const Pair& b) {
        if (a.v != b.v) return a.v > b.v;
        if (a.i != b.i) return a.i < b.i;
        return a.j < b.j;
    });
    std::vector<double> gx, gw;
    gauss_legendre(24, gx, gw);
    std::vector<double> inv(nm);
    for (int n = 0; n < nm; ++n) inv[n] = 1.0 / l2_norm_1d(om[n], om[n] / c, gx, gw);
    ctx->sqrt_lam.resize(K);
    ctx->om_x.resize(K); ctx->om_y.resize(K);
    ctx->amp_x.resize(K); ctx->amp_y.resize(K);
    ctx->inv_x.resize(K); ctx->inv_y.resize(K);
    std::vector<double> modes(7 * (size_t)K);
    for (int k = 0; k < K; ++k) {
        const Pair& q = all[k];
        ctx->sqrt_lam[k] = std::sqrt(p.sigma2 * q.v);
        ctx->om_x[k] = om[q.i]; ctx->om_y[k] = om[q.j];
        ctx->amp_x[k] = om[q.i] / c; ctx->amp_y[k] = om[q.j] / c;
        ctx->inv_x[k] = inv[q.i]; ctx->inv_y[k] = inv[q.j];
        double* m = &modes[7 * (size_t)k];
        m[0] = ctx->sqrt_lam[k]; m[1] = ctx->om_x[k]; m[2] = ctx->om_y[k];
        m[3] = ctx->amp_x[k]; m[4] = ctx->amp_y[k]; m[5] = ctx->inv_x[k]; m[6] = ctx->inv_y[k];
    }
    MLS_CHECK_HIP(hipMalloc(&ctx->d_modes, sizeof(double) * modes.size()));
    MLS_CHECK_HIP(hipMemcpy(ctx->d_modes, modes.data(), sizeof(double) * modes.size(),
                            hipMemcpyHostToDevice));
    const int Kp = (K + 31) / 32 * 32;
    for (int l = p.l_min; l <= p.l_max; ++l) {
        const int64_t ne = n_elem(l);
        MLS_CHECK_HIP(hipMalloc(&ctx->d_B[l], sizeof(double) * (size_t)K * ne));
        if (p.precision == MLS2MC_MIXED) {
            MLS_CHECK_HIP(hipMalloc(&ctx->d_B16[l], sizeof(__hip_bfloat16) * (size_t)Kp * ne));
            MLS_CHECK_HIP(hipMemset(ctx->d_B16[l], 0, sizeof(__hip_bfloat16) * (size_t)Kp * ne));
        }
        dim3 grid((unsigned)((ne + 255) / 256), (unsigned)K);
        kl_basis_kernel<<<grid, 256>>>(ctx->d_modes, K, l, ne, ctx->d_B[l], ctx->d_B16[l], Kp);
        MLS_CHECK_HIP(hipGetLastError());
    }
    MLS_CHECK_HIP(hipDeviceSynchronize());
    return MLS2MC_OK;
}

// ----------------------------------------------------------------- GEMM --
// FP64 on the matrix cores: v_mfma_f64_16x16x4f64.  A workgroup of four
// waves computes a 64 RT (particles) x 64 (elements) tile; wave w owns rows
// 16 RT w .. 16 RT (w + 1) - 1 in RT row tiles of 16, each with four 16x16
// accumulators.  Operand lanes: A[i][k] with i = lane%16, k = lane/16;
// B[k][j] with j = lane%16, k = lane/16.  Result: lane holds
// D[lane/16 + 4v][lane%16], v = 0..3 (FP64 accumulator layout).  The
// workgroup stages 16-deep k-chunks of its theta rows and 64 basis columns
// through LDS (coalesced loads, the next chunk prefetched into registers
// while the current one feeds the MFMAs), so a global round trip is paid
// once per 16 k instead of once per MFMA step.  With RT = 2 every basis
// operand read from LDS feeds two MFMAs and every staged basis chunk serves
// 128 particles; the per-element k order is the same for every RT, so the
// results are bitwise those of RT = 1.
constexpr int kGemmKC = 16;
template <int RT>
struct GemmF64SmemT {
    double a[64 * RT][kGemmKC + 1];  // theta rows x k (padded against bank conflicts)
    double b[kGemmKC][64 + 1];       // k x basis columns
};
using GemmF64Smem = GemmF64SmemT<1>;

template <bool EXP, int RT = 1>
__device__ __forceinline__ void gemm_f64_tile(const double* __restrict__ theta, const double* __restrict__ B,
                                              double* __restrict__ out, int64_t N, int K, int64_t ne,
                                              int64_t bx, int64_t by, GemmF64SmemT<RT>& sm)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int64_t e0 = bx * 64;
    const int64_t pb = by * 64 * RT;
    dbl4 acc[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[rt][c] = dbl4{0.0, 0.0, 0.0, 0.0};
    // each thread moves 4 RT theta and 4 basis values per chunk
    double ra[4 * RT], rb[4];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int t = 0; t < 4 * RT; ++t) {
            const int idx = tid + 256 * t;
            const int row = idx >> 4, kk = idx & 15;          // theta: 64 RT rows x 16 k
            const int k = kc + kk;
            ra[t] = (pb + row < N && k < K) ? theta[(pb + row) * K + k] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int idx = tid + 256 * t;
            const int kb = idx >> 6, col = idx & 63;         // basis: 16 k x 64 columns
            const int k2 = kc + kb;
            rb[t] = (k2 < K && e0 + col < ne) ? B[(int64_t)k2 * ne + e0 + col] : 0.0;
        }
    };
    fetch(0);
    for (int kc = 0; kc < K; kc += kGemmKC) {
        __syncthreads();  // the previous chunk's reads are done
#pragma unroll
        for (int t = 0; t < 4 * RT; ++t) {
            const int idx = tid + 256 * t;
            sm.a[idx >> 4][idx & 15] = ra[t];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int idx = tid + 256 * t;
            sm.b[idx >> 6][idx & 63] = rb[t];
        }
        __syncthreads();
        if (kc + kGemmKC < K) fetch(kc + kGemmKC);
#pragma unroll
        for (int ks = 0; ks < kGemmKC; ks += 4) {
            double a[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) a[rt] = sm.a[wv * 16 * RT + 16 * rt + r][ks + kq];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double b = sm.b[ks + kq][c * 16 + r];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    acc[rt][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt], b, acc[rt][c], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t p0 = pb + wv * 16 * RT + 16 * rt;
        // lane (r, kq) holds rows p0 + kq + 4 v of columns e0 + 16 c + r; a
        // block inside the output is stored without per-element tests and, as
        // in the BF16 kernels, non-temporally (the field is read once, after
        // the launch)
        if (p0 + 16 <= N && e0 + 64 <= ne) {
            double* o = out + (p0 + kq) * ne + e0 + r;
#pragma unroll
            for (int v = 0; v < 4; ++v, o += 4 * ne)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    __builtin_nontemporal_store(EXP ? exp(acc[rt][c][v]) : acc[rt][c][v], o + 16 * c);
            continue;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = p0 + kq + 4 * v, col = e0 + c * 16 + r;
                if (row < N && col < ne) out[row * ne + col] = EXP ? exp(acc[rt][c][v]) : acc[rt][c][v];
            }
    }
}

// Three waves per SIMD (at most 168 registers): the 128-particle tile then
// keeps its accumulators in VGPRs without spilling, and a third wave hides
// the epilogue's FP64 exp behind the other waves' MFMAs (same-box A/B at
// h = 1/512, K = 200, N = 2048: 9.9 ms with the compiler's two waves,
// 9.1 ms with three)
template <bool EXP, int RT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void kl_gemm_f64(const double* __restrict__ theta,
                                                   const double* __restrict__ B,
                                                   double* __restrict__ out, int64_t N, int K,
                                                   int64_t ne, const int64_t* __restrict__ N_dev)
{
    __shared__ GemmF64SmemT<RT> sm;
    if (N_dev) N = min(N, *N_dev);
    if ((int64_t)blockIdx.y * 64 * RT >= N) return;
    gemm_f64_tile<EXP, RT>(theta, B, out, N, K, ne, blockIdx.x, blockIdx.y, sm);
}

// BF16 on the matrix cores with FP32 accumulation: v_mfma_f32_16x16x32_bf16.
// Operand lanes: A[i][8*(lane/16) + 0..7] with i = lane%16 (theta rows,
// rounded to BF16); B^T[j][8*(lane/16) + 0..7] with j = lane%16 (the basis is
// stored transposed, n_e x Kp, K padded to 32 with zeros).  Output
// kappa = e^a in FP32 (kappa_of below).  Tile 64 x 64 as above.  The workgroup stages
// 128-deep k-chunks of its theta rows (rounded once) and basis columns in
// LDS, so K <= 128 takes a single global round trip.
constexpr int kBfKC = 128;
struct GemmBf16Smem {
    __bf16 a[64][kBfKC + 8];  // theta rows x k (row padding against bank conflicts)
    __bf16 b[64][kBfKC + 8];  // basis columns x k
};

// kappa = e^a in FP32 as 2^(a log2 e): one multiply and one v_exp_f32.
// Rounding a log2 e to FP32 moves the exponent by at most |a| 2^-23
// (relative), and v_exp_f32 adds about one unit in the last place, so
// log kappa is within |a| 2^-23 + 2^-23 of a: under 2e-6 at |a| <= 16,
// three orders below the BF16 rounding of the field it finishes.
__device__ __forceinline__ float kappa_of(float a)
{
    return __builtin_amdgcn_exp2f(a * 1.44269504088896341f);
}

// Stores a wave's 16 x 64 block of kappa: lane (r, kq) holds rows
// p0 + 4 kq + v of columns e0 + 16 c + r.  When the block lies inside the
// output (every row tile but a ragged last one), the stores go without
// per-element tests from one row pointer per v, and they are non-temporal:
// kappa is read once, by the solver's set-up after the launch, and at the
// large levels it is many times the size of the caches.
__device__ __forceinline__ void store_kappa_block(const flt4 (&acc)[4], float* __restrict__ out, int64_t p0,
                                                  int64_t e0, int64_t N, int64_t ne, int r, int kq)
{
    if (p0 + 16 <= N && e0 + 64 <= ne) {
        float* o = out + (p0 + 4 * kq) * ne + e0 + r;
#pragma unroll
        for (int v = 0; v < 4; ++v, o += ne)
#pragma unroll
            for (int c = 0; c < 4; ++c) __builtin_nontemporal_store(kappa_of(acc[c][v]), o + 16 * c);
        return;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = p0 + 4 * kq + v, col = e0 + c * 16 + r;
            if (row < N && col < ne) out[row * ne + col] = kappa_of(acc[c][v]);
        }
}

__device__ __forceinline__ void gemm_bf16_tile(const double* __restrict__ theta,
                                               const __hip_bfloat16* __restrict__ Bt, float* __restrict__ out,
                                               int64_t N, int K, int Kp, int64_t ne, int64_t bx, int64_t by,
                                               GemmBf16Smem& sm)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int64_t e0 = bx * 64;
    const int64_t pb = by * 64;
    const int64_t p0 = pb + wv * 16;
    flt4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = flt4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < Kp; kc += kBfKC) {
        __syncthreads();  // the previous chunk's reads are done
        // theta chunk: 64 rows x 128 k, 32 values per thread (a row is 128 threads)
#pragma unroll 8
        for (int t = 0; t < 32; ++t) {
            const int idx = tid + 256 * t;
            const int row = idx >> 7, kk = idx & 127;
            const int k = kc + kk;
            const float v = (pb + row < N && k < K) ? (float)theta[(pb + row) * K + k] : 0.f;
            sm.a[row][kk] = (__bf16)v;
        }
        // basis chunk: 64 columns x 128 k in 16-byte vectors, 4 per thread
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int idx = tid + 256 * t;
            const int col = idx >> 4, part = idx & 15;
            const int k = kc + 8 * part;
            bf16x8 v;
            if (e0 + col < ne && k < Kp) {
                v = *reinterpret_cast<const bf16x8*>(Bt + (e0 + col) * Kp + k);
            } else {
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = (__bf16)0.f;
            }
            *reinterpret_cast<bf16x8*>(&sm.b[col][8 * part]) = v;
        }
        __syncthreads();
        const int kend = Kp - kc < kBfKC ? Kp - kc : kBfKC;  // a multiple of 32
        for (int ks = 0; ks < kend; ks += 32) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sm.a[wv * 16 + r][ks + 8 * kq]);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sm.b[c * 16 + r][ks + 8 * kq]);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
            }
        }
    }
    store_kappa_block(acc, out, p0, e0, N, ne, r, kq);
}

__global__ __launch_bounds__(256) void kl_gemm_bf16(const double* __restrict__ theta,
                                                    const __hip_bfloat16* __restrict__ Bt,
                                                    float* __restrict__ out, int64_t N, int K,
                                                    int Kp, int64_t ne, const int64_t* __restrict__ N_dev)
{
    __shared__ __align__(16) GemmBf16Smem sm;
    if (N_dev) N = min(N, *N_dev);
    if ((int64_t)blockIdx.y * 64 >= N) return;
    gemm_bf16_tile(theta, Bt, out, N, K, Kp, ne, blockIdx.x, blockIdx.y, sm);
}

// The single-batch BF16 field.  theta is rounded to BF16 once, into an
// N x Kp array (K padded to 32 with zeros).  Each workgroup owns one
// 64-element column tile: it stages that tile of the transposed basis in
// LDS once, and each of its four waves walks its own 16-row slabs of theta
// (slabs w, w + 4, ...), loading a slab's operands straight from the BF16
// copy (under half a MiB at K = 200 and N = 1024, so it is read from the
// L2).  The basis fragments do not change from slab to slab, so the
// compiler keeps them in registers across the loop.  The basis is read
// from HBM once per launch instead of once per row tile, no barrier sits in
// the row loop, and the kernel is bound by writing kappa.  The MFMA lanes,
// the k order and the rounding are those of gemm_bf16_tile, so the results
// are bitwise the same.  NKS = Kp / 32 is a template constant so that a
// slab's operands are whole register arrays.
__global__ void theta_bf16_kernel(const double* __restrict__ theta, __bf16* __restrict__ t16, int64_t N, int K,
                                  int Kp)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * Kp) return;
    const int64_t q = t / Kp;
    const int k = (int)(t - q * Kp);
    t16[t] = (__bf16)(k < K ? (float)theta[q * K + k] : 0.f);
}

constexpr int kColsMaxKs = 8;  // Kp <= 256

template <int NKS>
__global__ __launch_bounds__(256) void kl_gemm_bf16_cols(const __bf16* __restrict__ t16,
                                                         const __hip_bfloat16* __restrict__ Bt,
                                                         float* __restrict__ out, int64_t N, int64_t ne,
                                                         const int64_t* __restrict__ N_dev)
{
    constexpr int Kp = 32 * NKS;
    constexpr int ld = Kp + 8;  // row padding against bank conflicts
    __shared__ __align__(16) __bf16 sb[64 * ld];  // 64 basis columns x Kp
    if (N_dev) N = min(N, *N_dev);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int64_t e0 = (int64_t)blockIdx.x * 64;
    constexpr int vk = Kp / 8;  // 16-byte vectors per row
    for (int idx = tid; idx < 64 * vk; idx += 256) {
        const int col = idx / vk, part = idx - col * vk;
        bf16x8 v;
        if (e0 + col < ne) {
            v = *reinterpret_cast<const bf16x8*>(Bt + (e0 + col) * Kp + 8 * part);
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = (__bf16)0.f;
        }
        *reinterpret_cast<bf16x8*>(sb + col * ld + 8 * part) = v;
    }
    __syncthreads();
    const int64_t nslab = (N + 15) / 16;
    auto load = [&](int64_t sl, bf16x8* a) {
        const int64_t row = sl * 16 + r;
        if (row < N) {
            const bf16x8* src = reinterpret_cast<const bf16x8*>(t16 + row * Kp + 8 * kq);
#pragma unroll
            for (int q = 0; q < NKS; ++q) a[q] = src[4 * q];
        } else {
#pragma unroll
            for (int q = 0; q < NKS; ++q)
#pragma unroll
                for (int u = 0; u < 8; ++u) a[q][u] = (__bf16)0.f;
        }
    };
    for (int64_t sl = wv; sl < nslab; sl += 4) {
        bf16x8 a[NKS];
        load(sl, a);
        flt4 acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NKS; ++q) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bf16x8 b = *reinterpret_cast<const bf16x8*>(sb + (c * 16 + r) * ld + 32 * q + 8 * kq);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[q], b, acc[c], 0, 0, 0);
            }
        }
        store_kappa_block(acc, out, sl * 16, e0, N, ne, r, kq);
    }
}

// Grouped launch: one 1-D grid over the 64x64 tiles of several items (each
// its own theta, level basis and output).
__global__ __launch_bounds__(256) void kl_gemm_list(const GemmItem* __restrict__ items, int n_items, int K,
                                                    int Kp, int bf16)
{
    __shared__ __align__(16) union {
        GemmF64Smem f;
        GemmBf16Smem b;
    } sm;
    const int64_t t = blockIdx.x;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    const GemmItem& it = items[lo];
    const int64_t lt = t - it.tile_base;
    const int64_t bx = lt % it.tiles_x, by = lt / it.tiles_x;
    if (bf16) gemm_bf16_tile(it.theta, it.B16, (float*)it.out, it.N, K, Kp, it.ne, bx, by, sm.b);
    else gemm_f64_tile<true>(it.theta, it.B, (double*)it.out, it.N, K, it.ne, bx, by, sm.f);
}

int launch_kl_list(mls2mc_ctx* ctx, const GemmItem* items_dev, int n_items, int64_t total_tiles, hipStream_t s)
{
    if (total_tiles == 0) return MLS2MC_OK;
    MLS_REQUIRE(total_tiles < (int64_t(1) << 31), "kl_gemm_list: too many tiles");
    const bool mixed = ctx->prob.precision == MLS2MC_MIXED;
    const int K = ctx->prob.K, Kp = (K + 31) / 32 * 32;
    kl_gemm_list<<<(unsigned)total_tiles, 256, 0, s>>>(items_dev, n_items, K, Kp, mixed ? 1 : 0);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

int launch_kl_field(mls2mc_ctx* ctx, int l, int64_t N, const double* theta, void* out, int kind,
                    hipStream_t s, const int64_t* N_dev)
{
    if (N == 0) return MLS2MC_OK;
    const int64_t ne = n_elem(l);
    const int K = ctx->prob.K;
    MLS_REQUIRE((N + 63) / 64 <= 65535, "kl_field: N too large for one launch");
    dim3 grid((unsigned)((ne + 63) / 64), (unsigned)((N + 63) / 64));
    // FP64: 128-particle tiles once there are more than 64 particles
    dim3 grid2((unsigned)((ne + 63) / 64), (unsigned)((N + 127) / 128));
    ProfRec rec;
    if (ctx->prof_on) MLS_TRY(prof_begin(ctx, MLS2MC_PROF_GEMM, l, N, s, &rec));
    if (kind == MLS2MC_FIELD_LOG_F64 || kind == MLS2MC_FIELD_KAPPA_F64) {
        const double* Bl = ctx->d_B[l];
        double* o = (double*)out;
        const bool e = kind == MLS2MC_FIELD_KAPPA_F64;
        if (N <= 64) {
            if (e) kl_gemm_f64<true, 1><<<grid, 256, 0, s>>>(theta, Bl, o, N, K, ne, N_dev);
            else kl_gemm_f64<false, 1><<<grid, 256, 0, s>>>(theta, Bl, o, N, K, ne, N_dev);
        } else {
            if (e) kl_gemm_f64<true, 2><<<grid2, 256, 0, s>>>(theta, Bl, o, N, K, ne, N_dev);
            else kl_gemm_f64<false, 2><<<grid2, 256, 0, s>>>(theta, Bl, o, N, K, ne, N_dev);
        }
    } else if (kind == MLS2MC_FIELD_KAPPA_F32) {
        MLS_REQUIRE(ctx->d_B16[l] != nullptr, "kl_field: BF16 basis needs precision MIXED");
        const int Kp = (K + 31) / 32 * 32;
        if (Kp <= 32 * kColsMaxKs) {  // theta in BF16 once, then one workgroup per column tile
            MLS_TRY(ctx->ws_theta16.ensure(sizeof(__bf16) * (size_t)N * Kp));
            __bf16* t16 = ctx->ws_theta16.as<__bf16>();
            theta_bf16_kernel<<<(unsigned)((N * Kp + 255) / 256), 256, 0, s>>>(theta, t16, N, K, Kp);
            MLS_CHECK_HIP(hipGetLastError());
            const unsigned g = (unsigned)((ne + 63) / 64);
            float* o = (float*)out;
            const __hip_bfloat16* B16 = ctx->d_B16[l];
            switch (Kp / 32) {
            case 1: kl_gemm_bf16_cols<1><<<g, 256, 0, s>>>(t16, B16, o, N, ne, N_dev); break;
            case 2: kl_gemm_bf16_cols<2><<<g, 256, 0, s>>>(t16, B16, o, N, ne, N_dev); break;
            case 3: kl_gemm_bf16_cols<3><<<g, 256, 0, s>>>(t16, B16, o, N, ne, N_dev); break;
            case 4: kl_gemm_bf16_cols<4><<<g, 256, 0, s>>>(t16, B16, o, N, ne, N_dev); break;
            case 5: kl_gemm_bf16_cols<5><<<g, 256, 0, s>>>(t16, B16, o, N, ne, N_dev); break;
            case 6: kl_gemm_bf16_cols<6><<<g, 256, 0, s>>>(t16, B16, o, N, ne, N_dev); break;
            case 7: kl_gemm_bf16_cols<7><<<g, 256, 0, s>>>(t16, B16, o, N, ne, N_dev); break;
            default: kl_gemm_bf16_cols<8><<<g, 256, 0, s>>>(t16, B16, o, N, ne, N_dev); break;
            }
        } else {
            kl_gemm_bf16<<<grid, 256, 0, s>>>(theta, ctx->d_B16[l], (float*)out, N, K, Kp, ne, N_dev);
        }
    } else {
        MLS_REQUIRE(false, "kl_field: unknown output kind");
    }
    MLS_CHECK_HIP(hipGetLastError());
    if (ctx->prof_on) MLS_TRY(prof_end(ctx, MLS2MC_PROF_GEMM, l, rec, s));
    return MLS2MC_OK;
}

}  // namespace mls
