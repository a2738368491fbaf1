// Learned surrogate theta -> G_l(theta): an MLP K -> H -> H -> N_obs with
// erf-GELU, trained on the GPU from (theta, G_l(theta)) pairs the sampler
// produces, and used as the first stage of delayed-acceptance pCN (two-stage
// Metropolis-Hastings: the surrogate screens proposals, the FEM solve judges
// the survivors).  Matrix products run on the CDNA4 matrix cores as BF16
// MFMA with FP32 accumulation; master weights and Adam moments are FP32.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <random>

#include "common.h"

namespace mls {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ GEMM --
// C[M x N] = sum_k A(m,k) B(k,n) with A(m,k) = TA ? A[k lda + m] : A[m lda + k]
// and B(k,n) = TB ? B[n ldb + k] : B[k ldb + n]; operands are rounded to
// BF16 as the fragments are loaded (v_mfma_f32_16x16x32_bf16 lanes: A rows
// lane%16, k = 8(lane/16)+0..7; B cols lane%16, same k; D[4(lane/16)+v][lane%16]).
// Epilogues: 0 store; 1 +bias, store Z to C and GELU(Z) to C2; 2 +bias;
// 3 multiply by GELU'(Zin[m][n]) (backward through the activation); 4 store,
// and (TA only) also write the row sums over k of A, sum_k A(m,k), to C2[m]:
// the bias gradient of a layer comes out of its weight-gradient product.
enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_BIAS = 2, EPI_DGELU = 3, EPI_STORE_ASUM = 4 };

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
}

// Each wave owns one 16x16 tile of C, a workgroup 32x32.  The k loop loads
// the fragments of MLP_U consecutive 32-wide k steps before it issues their
// MFMAs, so one round of memory latency covers MLP_U steps (K <= 256 in the
// surrogate: at most two rounds).
constexpr int MLP_U = 4;

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void mlp_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                                const float* __restrict__ B, int ldb,
                                                const float* __restrict__ bias, float* __restrict__ C,
                                                float* __restrict__ C2, const float* __restrict__ Zin,
                                                int ldc)
{
    static_assert(EPI != EPI_STORE_ASUM || TA, "row sums of A are taken for the transposed-A form");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int m0 = blockIdx.y * 32 + 16 * (wv >> 1);
    const int n0 = blockIdx.x * 32 + 16 * (wv & 1);
    const bool asum = EPI == EPI_STORE_ASUM && blockIdx.x == 0 && (wv & 1) == 0;
    flt4 acc = {0.f, 0.f, 0.f, 0.f};
    float rs = 0.f;
    const int am = m0 + r, bn = n0 + r;
    for (int k0 = 0; k0 < K; k0 += 32 * MLP_U) {
        bf16x8 a[MLP_U], b[MLP_U];
#pragma unroll
        for (int u = 0; u < MLP_U; ++u) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int k = k0 + 32 * u + 8 * kq + t;
                float av = 0.f, bv = 0.f;
                if (am < M && k < K) av = TA ? A[(int64_t)k * lda + am] : A[(int64_t)am * lda + k];
                if (bn < N && k < K) bv = TB ? B[(int64_t)bn * ldb + k] : B[(int64_t)k * ldb + bn];
                if (EPI == EPI_STORE_ASUM) rs += av;
                a[u][t] = (__bf16)av;
                b[u][t] = (__bf16)bv;
            }
        }
#pragma unroll
        for (int u = 0; u < MLP_U; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], b[u], acc, 0, 0, 0);
    }
    if (EPI == EPI_STORE_ASUM) {
        // lanes r, r+16, r+32, r+48 hold the partial sums of row am
        rs += __shfl_xor(rs, 16);
        rs += __shfl_xor(rs, 32);
        if (asum && kq == 0 && am < M) C2[am] = rs;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int m = m0 + 4 * kq + v, n = n0 + r;
        if (m >= M || n >= N) continue;
        float z = acc[v];
        const int64_t o = (int64_t)m * ldc + n;
        if (EPI == EPI_BIAS_GELU) {
            z += bias[n];
            C[o] = z;
            C2[o] = gelu(z);
        } else if (EPI == EPI_BIAS) {
            C[o] = z + bias[n];
        } else if (EPI == EPI_DGELU) {
            C[o] = z * gelu_d(Zin[o]);
        } else {
            C[o] = z;
        }
    }
}

template <bool TA, bool TB, int EPI>
static int gemm(int M, int N, int K, const float* A, int lda, const float* B, int ldb, const float* bias,
                float* C, float* C2, const float* Zin, int ldc, hipStream_t s)
{
    if (M == 0 || N == 0) return MLS2MC_OK;
    dim3 grid((unsigned)((N + 31) / 32), (unsigned)((M + 31) / 32));
    mlp_gemm<TA, TB, EPI><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, bias, C, C2, Zin, ldc);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// ------------------------------------------------------- small kernels --
// delta = (out - t) * scale, loss = scale * sum (out - t)^2 / 2 (one workgroup)
__global__ __launch_bounds__(1024) void loss_delta_kernel(int64_t n, const float* __restrict__ out,
                                                          const float* __restrict__ t, float scale,
                                                          float* __restrict__ delta, float* __restrict__ loss)
{
    __shared__ double red[16];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const float d = out[i] - t[i];
        delta[i] = d * scale;
        s += 0.5 * (double)d * (double)d;
    }
    s = block_sum<1024>(s, red);
    if (threadIdx.x == 0) loss[0] = (float)(s * scale);
}

__global__ void adam_kernel(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                            float c1, float c2, float eps)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// rows idx[b] (or b) of a double matrix, standardised, to float
__global__ void standardize_kernel(int64_t B, int D, const int32_t* __restrict__ idx,
                                   const double* __restrict__ src, const float* __restrict__ mu,
                                   const float* __restrict__ sd, float* __restrict__ dst)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= B * D) return;
    const int64_t b = t / D;
    const int k = (int)(t - b * D);
    const int64_t row = idx ? idx[b] : b;
    const double v = src[row * D + k];
    dst[t] = mu ? (float)((v - (double)mu[k]) / (double)sd[k]) : (float)v;
}

__global__ void unstandardize_kernel(int64_t B, int O, const float* __restrict__ out,
                                     const float* __restrict__ mu, const float* __restrict__ sd,
                                     double* __restrict__ G)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= B * O) return;
    const int o = (int)(t % O);
    G[t] = (double)mu[o] + (double)sd[o] * (double)out[t];
}

// column mean and standard deviation of an n x D double matrix (one block per column)
__global__ __launch_bounds__(256) void col_stats_kernel(int64_t n, int D, const double* __restrict__ X,
                                                        float* __restrict__ mu, float* __restrict__ sd)
{
    __shared__ double red[4];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += X[i * D + k];
    const double mean = block_sum<256>(s, red) / (double)n;
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double d = X[i * D + k] - mean;
        q += d * d;
    }
    const double var = block_sum<256>(q, red) / (double)n;
    if (threadIdx.x == 0) {
        mu[k] = (float)mean;
        sd[k] = (float)(var > 1e-30 ? sqrt(var) : 1.0);
    }
}

__global__ void f2d_kernel(int64_t n, const float* __restrict__ a, double* __restrict__ b)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

__global__ void f2f_scaled_kernel(int64_t n, const double* __restrict__ z, float scale, float* __restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = scale * (float)z[i];
}

// ----------------------------------------------------------- surrogate --
struct Surrogate {
    int D = 0, H = 0, O = 0;
    int64_t np = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float *mu_x = nullptr, *sd_x = nullptr, *mu_y = nullptr, *sd_y = nullptr;
    int64_t adam_t = 0;
    bool standardized = false;
    // dataset ring
    int64_t cap = 0, count = 0, head = 0;
    double *ds_th = nullptr, *ds_G = nullptr;
    // activations for up to bmax rows
    int64_t bmax = 0;
    float *X = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *OUT = nullptr;
    float *T = nullptr, *D3 = nullptr, *D2 = nullptr, *D1 = nullptr, *loss = nullptr;
    int32_t* perm = nullptr;
    float* W1() const { return p; }
    float* b1() const { return p + (int64_t)H * D; }
    float* W2() const { return b1() + H; }
    float* b2() const { return W2() + (int64_t)H * H; }
    float* W3() const { return b2() + H; }
    float* b3() const { return W3() + (int64_t)O * H; }
};

static void sur_free(Surrogate* S)
{
    void* ptrs[] = {S->p, S->g, S->m, S->v, S->mu_x, S->sd_x, S->mu_y, S->sd_y, S->ds_th, S->ds_G,
                    S->X, S->Z1, S->H1, S->Z2, S->H2, S->OUT, S->T, S->D3, S->D2, S->D1, S->loss, S->perm};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    *S = Surrogate();
}

void surrogate_destroy(mls2mc_ctx* ctx)
{
    if (ctx->sur) {
        sur_free(ctx->sur);
        delete ctx->sur;
        ctx->sur = nullptr;
    }
}

static int sur_ensure_batch(Surrogate* S, int64_t B)
{
    if (B <= S->bmax) return MLS2MC_OK;
    float** acts[] = {&S->X, &S->Z1, &S->H1, &S->Z2, &S->H2, &S->OUT, &S->T, &S->D3, &S->D2, &S->D1};
    for (float** a : acts)
        if (*a) { (void)hipFree(*a); *a = nullptr; }
    const int64_t w = std::max<int64_t>(std::max(S->D, S->H), S->O);
    for (float** a : acts) MLS_CHECK_HIP(hipMalloc(a, sizeof(float) * (size_t)B * w));
    S->bmax = B;
    return MLS2MC_OK;
}

// forward of B standardised rows in S->X; outputs in S->OUT (standardised)
static int sur_forward(Surrogate* S, int64_t B, hipStream_t s)
{
    const int D = S->D, H = S->H, O = S->O;
    MLS_TRY((gemm<false, true, EPI_BIAS_GELU>((int)B, H, D, S->X, D, S->W1(), D, S->b1(), S->Z1, S->H1, nullptr, H, s)));
    MLS_TRY((gemm<false, true, EPI_BIAS_GELU>((int)B, H, H, S->H1, H, S->W2(), H, S->b2(), S->Z2, S->H2, nullptr, H, s)));
    MLS_TRY((gemm<false, true, EPI_BIAS>((int)B, O, H, S->H2, H, S->W3(), H, S->b3(), S->OUT, nullptr, nullptr, O, s)));
    return MLS2MC_OK;
}

// gradient of mean (out - t)^2 / 2 w.r.t. all parameters into S->g; T holds targets
static int sur_backward(Surrogate* S, int64_t B, hipStream_t s)
{
    const int D = S->D, H = S->H, O = S->O;
    const float scale = 1.0f / (float)(B * O);
    loss_delta_kernel<<<1, 1024, 0, s>>>(B * O, S->OUT, S->T, scale, S->D3, S->loss);
    MLS_CHECK_HIP(hipGetLastError());
    float *gW1 = S->g, *gb1 = gW1 + (int64_t)H * D, *gW2 = gb1 + H, *gb2 = gW2 + (int64_t)H * H,
          *gW3 = gb2 + H, *gb3 = gW3 + (int64_t)O * H;
    // layer 3: dW3 = D3^T H2 and db3 = colsum D3 in one product; dH2 = D3 W3 (then * GELU'(Z2))
    MLS_TRY((gemm<true, false, EPI_STORE_ASUM>(O, H, (int)B, S->D3, O, S->H2, H, nullptr, gW3, gb3, nullptr, H, s)));
    MLS_TRY((gemm<false, false, EPI_DGELU>((int)B, H, O, S->D3, O, S->W3(), H, nullptr, S->D2, nullptr, S->Z2, H, s)));
    // layer 2
    MLS_TRY((gemm<true, false, EPI_STORE_ASUM>(H, H, (int)B, S->D2, H, S->H1, H, nullptr, gW2, gb2, nullptr, H, s)));
    MLS_TRY((gemm<false, false, EPI_DGELU>((int)B, H, H, S->D2, H, S->W2(), H, nullptr, S->D1, nullptr, S->Z1, H, s)));
    // layer 1
    MLS_TRY((gemm<true, false, EPI_STORE_ASUM>(H, D, (int)B, S->D1, H, S->X, D, nullptr, gW1, gb1, nullptr, D, s)));
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// ------------------------------------------------ delayed acceptance --
// stage-1 potential of the surrogate: beta * Phi(G~)
__global__ void da_psis_kernel(int64_t N, int nobs, const double* __restrict__ Gs, const double* __restrict__ y,
                               double inv_sigma, double beta, double* __restrict__ psis)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= N) return;
    double s = 0.0;
    for (int o = 0; o < nobs; ++o) {
        const double r = (y[o] - Gs[j * nobs + o]) * inv_sigma;
        s += r * r;
    }
    psis[j] = beta * 0.5 * s;
}

// Stage 1 and compaction in one workgroup: thread k owns the contiguous chunk
// [k N / BS, (k+1) N / BS); survivors keep their ascending order in idx.
__global__ __launch_bounds__(1024) void da_stage1_kernel(int64_t N, const double* __restrict__ u1,
                                                         const double* __restrict__ ps_old,
                                                         const double* __restrict__ ps_new,
                                                         int32_t* __restrict__ idx, int64_t* __restrict__ count,
                                                         uint8_t* __restrict__ acc, uint8_t* __restrict__ pass1,
                                                         int64_t* __restrict__ n_lo, int64_t* __restrict__ n_hi)
{
    __shared__ int64_t part[1024];
    const int64_t lo = (int64_t)threadIdx.x * N / 1024, hi = (int64_t)(threadIdx.x + 1) * N / 1024;
    int64_t c = 0;
    for (int64_t j = lo; j < hi; ++j) {
        const bool s1 = log(u1[j]) < -(ps_new[j] - ps_old[j]);
        c += s1 ? 1 : 0;
        acc[j] = 0;
        if (pass1) pass1[j] = s1 ? 1 : 0;
    }
    part[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t a = 0;
        for (int k = 0; k < 1024; ++k) {
            const int64_t v = part[k];
            part[k] = a;
            a += v;
        }
        count[0] = a;
        if (n_lo) n_lo[0] += a;
        if (n_hi) n_hi[0] += a;
    }
    __syncthreads();
    int64_t o = part[threadIdx.x];
    for (int64_t j = lo; j < hi; ++j)
        if (log(u1[j]) < -(ps_new[j] - ps_old[j])) idx[o++] = (int32_t)j;
}

__global__ void gather_count_kernel(int64_t N, int ncols, const int32_t* __restrict__ idx,
                                    const int64_t* __restrict__ count, const double* __restrict__ src,
                                    double* __restrict__ dst)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t c = t / ncols;
    if (c >= N || c >= count[0]) return;
    const int k = (int)(t - c * ncols);
    dst[t] = src[(int64_t)idx[c] * ncols + k];
}

// Error of the surrogate against the FEM solve that judges it in stage 2:
// e_c = ||G~(theta'_j) - G(theta'_j)||_2 / sigma_n for the survivors c <
// count (j = idx[c]); acc[0] += sum e, acc[1] = max(acc[1], max e),
// acc[2] += number of survivors.  One workgroup, deterministic sums.
__global__ __launch_bounds__(256) void da_err_kernel(int64_t N, const int64_t* __restrict__ count,
                                                     const int32_t* __restrict__ idx, int nobs,
                                                     const double* __restrict__ Gs, const double* __restrict__ Gf,
                                                     double inv_sigma, double* __restrict__ acc)
{
    __shared__ double red[4];
    const int64_t n = count[0] < N ? count[0] : N;
    double sum = 0.0, mx = 0.0;
    for (int64_t c = threadIdx.x; c < n; c += 256) {
        const int64_t j = idx[c];
        double e2 = 0.0;
        for (int o = 0; o < nobs; ++o) {
            const double d = Gs[j * nobs + o] - Gf[c * nobs + o];
            e2 += d * d;
        }
        const double e = sqrt(e2) * inv_sigma;
        sum += e;
        mx = fmax(mx, e);
    }
    sum = block_sum<256>(sum, red);
    mx = block_max<256>(mx, red);
    if (threadIdx.x == 0) {
        acc[0] += sum;
        acc[1] = fmax(acc[1], mx);
        acc[2] += (double)n;
    }
}

// stage 2 for the survivors: Psi of the FEM solve corrected by the surrogate
__global__ void da_stage2_kernel(int64_t N, const int64_t* __restrict__ count, const int32_t* __restrict__ idx,
                                 int K, int nobs, int mode, double beta, double zeta,
                                 const double* __restrict__ u2, const double* __restrict__ ps_old,
                                 const double* __restrict__ ps_new, const double* __restrict__ thn,
                                 const double* __restrict__ Gcl, const double* __restrict__ Gch,
                                 const double* __restrict__ pcl, const double* __restrict__ pch,
                                 const int8_t* __restrict__ stl, const int8_t* __restrict__ sth,
                                 double* __restrict__ th, double* __restrict__ Gl, double* __restrict__ Gh,
                                 double* __restrict__ pl, double* __restrict__ ph, uint8_t* __restrict__ acc)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= N || c >= count[0]) return;
    const int64_t j = idx[c];
    const bool need_lo = mode != 2, need_hi = mode != 0;
    double po, pn;
    if (mode == 0) {
        po = beta * pl[j];
        pn = beta * pcl[c];
    } else if (mode == 1) {
        po = beta * ((1.0 - zeta) * pl[j] + zeta * ph[j]);
        pn = beta * ((1.0 - zeta) * pcl[c] + zeta * pch[c]);
    } else {
        po = beta * ph[j];
        pn = beta * pch[c];
    }
    bool ok = true;
    if (need_lo && stl[c] != 0) ok = false;
    if (need_hi && sth[c] != 0) ok = false;
    const bool a = ok && (log(u2[j]) < -(pn - po) + (ps_new[j] - ps_old[j]));
    if (!a) return;
    for (int k = 0; k < K; ++k) th[j * K + k] = thn[j * K + k];
    if (need_lo) {
        for (int o = 0; o < nobs; ++o) Gl[j * nobs + o] = Gcl[c * nobs + o];
        pl[j] = pcl[c];
    }
    if (need_hi) {
        for (int o = 0; o < nobs; ++o) Gh[j * nobs + o] = Gch[c * nobs + o];
        ph[j] = pch[c];
    }
    acc[j] = 1;
}

}  // namespace mls

using namespace mls;

extern "C" {

int mls2mc_surrogate_init(mls2mc_ctx* ctx, int hidden, int64_t capacity, uint64_t seed, void* stream)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(hidden >= 16 && hidden <= 1024 && hidden % 16 == 0, "surrogate_init: hidden must be a multiple of 16 in [16, 1024]");
    MLS_REQUIRE(capacity >= 1 && capacity <= (int64_t(1) << 24), "surrogate_init: capacity in [1, 2^24]");
    const hipStream_t s = (hipStream_t)stream;
    surrogate_destroy(ctx);
    ctx->sur = new Surrogate();
    Surrogate* S = ctx->sur;
    S->D = ctx->prob.K;
    S->H = hidden;
    S->O = ctx->nobs;
    const int D = S->D, H = S->H, O = S->O;
    S->np = (int64_t)H * D + H + (int64_t)H * H + H + (int64_t)O * H + O;
    for (float** a : {&S->p, &S->g, &S->m, &S->v}) MLS_CHECK_HIP(hipMalloc(a, sizeof(float) * S->np));
    for (float** a : {&S->mu_x, &S->sd_x}) MLS_CHECK_HIP(hipMalloc(a, sizeof(float) * D));
    for (float** a : {&S->mu_y, &S->sd_y}) MLS_CHECK_HIP(hipMalloc(a, sizeof(float) * O));
    MLS_CHECK_HIP(hipMalloc(&S->loss, sizeof(float) * 4));
    S->cap = capacity;
    MLS_CHECK_HIP(hipMalloc(&S->ds_th, sizeof(double) * (size_t)capacity * D));
    MLS_CHECK_HIP(hipMalloc(&S->ds_G, sizeof(double) * (size_t)capacity * O));
    MLS_CHECK_HIP(hipMalloc(&S->perm, sizeof(int32_t) * (size_t)capacity));
    // He initialisation from Philox normals; zero biases and moments
    MLS_CHECK_HIP(hipMemsetAsync(S->p, 0, sizeof(float) * S->np, s));
    MLS_CHECK_HIP(hipMemsetAsync(S->m, 0, sizeof(float) * S->np, s));
    MLS_CHECK_HIP(hipMemsetAsync(S->v, 0, sizeof(float) * S->np, s));
    DevBuf z;
    MLS_TRY(z.ensure(sizeof(double) * (size_t)std::max<int64_t>((int64_t)H * std::max(D, H), (int64_t)O * H)));
    struct { float* w; int64_t n; int fan; } L[3] = {{S->W1(), (int64_t)H * D, D}, {S->W2(), (int64_t)H * H, H},
                                                      {S->W3(), (int64_t)O * H, H}};
    for (int q = 0; q < 3; ++q) {
        MLS_TRY(launch_philox(seed, 7, 0, (uint32_t)q, L[q].n, 1, z.as<double>(), s));
        f2f_scaled_kernel<<<(unsigned)((L[q].n + 255) / 256), 256, 0, s>>>(L[q].n, z.as<double>(),
                                                                         std::sqrt(2.0f / L[q].fan), L[q].w);
        MLS_CHECK_HIP(hipGetLastError());
    }
    MLS_CHECK_HIP(hipStreamSynchronize(s));
    z.release();
    return MLS2MC_OK;
}

int mls2mc_surrogate_n_params(const mls2mc_ctx* ctx)
{
    return (ctx && ctx->sur) ? (int)ctx->sur->np : -1;
}

int mls2mc_surrogate_set_params(mls2mc_ctx* ctx, const float* params, void* stream)
{
    MLS_REQUIRE(ctx && ctx->sur && params, "surrogate_set_params: no surrogate or null pointer");
    MLS_CHECK_HIP(hipMemcpyAsync(ctx->sur->p, params, sizeof(float) * ctx->sur->np, hipMemcpyDeviceToDevice,
                                 (hipStream_t)stream));
    return MLS2MC_OK;
}

int mls2mc_surrogate_get_params(mls2mc_ctx* ctx, float* params, void* stream)
{
    MLS_REQUIRE(ctx && ctx->sur && params, "surrogate_get_params: no surrogate or null pointer");
    MLS_CHECK_HIP(hipMemcpyAsync(params, ctx->sur->p, sizeof(float) * ctx->sur->np, hipMemcpyDeviceToDevice,
                                 (hipStream_t)stream));
    return MLS2MC_OK;
}

int mls2mc_surrogate_add_pairs(mls2mc_ctx* ctx, int64_t n, const double* theta, const double* G, void* stream)
{
    MLS_REQUIRE(ctx && ctx->sur, "surrogate_add_pairs: call mls2mc_surrogate_init first");
    MLS_REQUIRE(n >= 0, "surrogate_add_pairs: n < 0");
    if (n == 0) return MLS2MC_OK;
    MLS_REQUIRE(theta && G, "surrogate_add_pairs: null pointer");
    Surrogate* S = ctx->sur;
    const hipStream_t s = (hipStream_t)stream;
    if (n > S->cap) {  // keep the last cap pairs
        theta += (n - S->cap) * S->D;
        G += (n - S->cap) * S->O;
        n = S->cap;
    }
    int64_t done = 0;
    while (done < n) {
        const int64_t k = std::min(n - done, S->cap - S->head);
        MLS_CHECK_HIP(hipMemcpyAsync(S->ds_th + S->head * S->D, theta + done * S->D, sizeof(double) * k * S->D,
                                     hipMemcpyDeviceToDevice, s));
        MLS_CHECK_HIP(hipMemcpyAsync(S->ds_G + S->head * S->O, G + done * S->O, sizeof(double) * k * S->O,
                                     hipMemcpyDeviceToDevice, s));
        S->head = (S->head + k) % S->cap;
        done += k;
    }
    S->count = std::min(S->cap, S->count + n);
    return MLS2MC_OK;
}

int64_t mls2mc_surrogate_n_pairs(const mls2mc_ctx* ctx) { return (ctx && ctx->sur) ? ctx->sur->count : -1; }

int mls2mc_surrogate_train(mls2mc_ctx* ctx, int epochs, int batch, double lr, uint64_t seed, float* loss_out,
                           void* stream)
{
    MLS_REQUIRE(ctx && ctx->sur, "surrogate_train: call mls2mc_surrogate_init first");
    Surrogate* S = ctx->sur;
    MLS_REQUIRE(epochs >= 0 && batch >= 1 && batch <= 65536 && lr > 0, "surrogate_train: bad epochs/batch/lr");
    MLS_REQUIRE(S->count >= batch, "surrogate_train: fewer pairs than one batch");
    const hipStream_t s = (hipStream_t)stream;
    MLS_TRY(sur_ensure_batch(S, batch));
    const int64_t n = S->count;
    // standardisation statistics of the current dataset
    col_stats_kernel<<<S->D, 256, 0, s>>>(n, S->D, S->ds_th, S->mu_x, S->sd_x);
    col_stats_kernel<<<S->O, 256, 0, s>>>(n, S->O, S->ds_G, S->mu_y, S->sd_y);
    MLS_CHECK_HIP(hipGetLastError());
    S->standardized = true;
    std::mt19937_64 gen(seed);
    std::vector<int32_t> perm(n);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const int64_t nb = n / batch;
    for (int ep = 0; ep < epochs; ++ep) {
        std::iota(perm.begin(), perm.end(), 0);
        std::shuffle(perm.begin(), perm.end(), gen);
        MLS_CHECK_HIP(hipMemcpyAsync(S->perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        double ep_loss = 0.0;
        for (int64_t bi = 0; bi < nb; ++bi) {
            const int32_t* idx = S->perm + bi * batch;
            standardize_kernel<<<(unsigned)((batch * S->D + 255) / 256), 256, 0, s>>>(batch, S->D, idx, S->ds_th,
                                                                                     S->mu_x, S->sd_x, S->X);
            standardize_kernel<<<(unsigned)((batch * S->O + 255) / 256), 256, 0, s>>>(batch, S->O, idx, S->ds_G,
                                                                                     S->mu_y, S->sd_y, S->T);
            MLS_CHECK_HIP(hipGetLastError());
            MLS_TRY(sur_forward(S, batch, s));
            MLS_TRY(sur_backward(S, batch, s));
            ++S->adam_t;
            const float c1 = 1.f - std::pow(b1, (float)S->adam_t), c2 = 1.f - std::pow(b2, (float)S->adam_t);
            adam_kernel<<<(unsigned)((S->np + 255) / 256), 256, 0, s>>>(S->np, S->p, S->g, S->m, S->v, (float)lr,
                                                                        b1, b2, c1, c2, eps);
            MLS_CHECK_HIP(hipGetLastError());
            if (bi == nb - 1 && loss_out) {
                float l;
                MLS_CHECK_HIP(hipMemcpyAsync(&l, S->loss, sizeof(float), hipMemcpyDeviceToHost, s));
                MLS_CHECK_HIP(hipStreamSynchronize(s));
                ep_loss = l;
            }
        }
        if (loss_out) loss_out[ep] = (float)ep_loss;
    }
    return MLS2MC_OK;
}

int mls2mc_surrogate_predict(mls2mc_ctx* ctx, int64_t N, const double* theta, double* G_out, void* stream)
{
    MLS_REQUIRE(ctx && (ctx->sur || ctx->d_sur_S), "surrogate_predict: call mls2mc_surrogate_init first");
    MLS_REQUIRE(N >= 0, "surrogate_predict: N < 0");
    if (N == 0) return MLS2MC_OK;
    MLS_REQUIRE(theta && G_out, "surrogate_predict: null pointer");
    if (ctx->d_sur_S)  // the linear surrogate
        return launch_linear_map(N, ctx->prob.K, ctx->nobs, ctx->d_sur_S, theta, G_out, (hipStream_t)stream);
    Surrogate* S = ctx->sur;
    const hipStream_t s = (hipStream_t)stream;
    const int64_t chunk = 4096;
    MLS_TRY(sur_ensure_batch(S, std::min(N, chunk)));
    for (int64_t q0 = 0; q0 < N; q0 += chunk) {
        const int64_t B = std::min(chunk, N - q0);
        standardize_kernel<<<(unsigned)((B * S->D + 255) / 256), 256, 0, s>>>(
            B, S->D, nullptr, theta + q0 * S->D, S->standardized ? S->mu_x : nullptr, S->sd_x, S->X);
        MLS_CHECK_HIP(hipGetLastError());
        MLS_TRY(sur_forward(S, B, s));
        if (S->standardized) {
            unstandardize_kernel<<<(unsigned)((B * S->O + 255) / 256), 256, 0, s>>>(B, S->O, S->OUT, S->mu_y,
                                                                                   S->sd_y, G_out + q0 * S->O);
        } else {
            f2d_kernel<<<(unsigned)((B * S->O + 255) / 256), 256, 0, s>>>(B * S->O, S->OUT, G_out + q0 * S->O);
        }
        MLS_CHECK_HIP(hipGetLastError());
    }
    return MLS2MC_OK;
}

// loss and gradient on raw (unstandardised) inputs and targets, for checks
int mls2mc_surrogate_loss_grad(mls2mc_ctx* ctx, int64_t B, const double* x, const double* target, float* loss_out,
                               float* grad_out, void* stream)
{
    MLS_REQUIRE(ctx && ctx->sur, "surrogate_loss_grad: call mls2mc_surrogate_init first");
    MLS_REQUIRE(B >= 1 && B <= 65536, "surrogate_loss_grad: need 1 <= B <= 65536");
    MLS_REQUIRE(x && target && loss_out && grad_out, "surrogate_loss_grad: null pointer");
    Surrogate* S = ctx->sur;
    const hipStream_t s = (hipStream_t)stream;
    MLS_TRY(sur_ensure_batch(S, B));
    standardize_kernel<<<(unsigned)((B * S->D + 255) / 256), 256, 0, s>>>(B, S->D, nullptr, x, nullptr, nullptr, S->X);
    standardize_kernel<<<(unsigned)((B * S->O + 255) / 256), 256, 0, s>>>(B, S->O, nullptr, target, nullptr, nullptr, S->T);
    MLS_CHECK_HIP(hipGetLastError());
    MLS_TRY(sur_forward(S, B, s));
    MLS_TRY(sur_backward(S, B, s));
    MLS_CHECK_HIP(hipMemcpyAsync(grad_out, S->g, sizeof(float) * S->np, hipMemcpyDeviceToDevice, s));
    MLS_CHECK_HIP(hipMemcpyAsync(loss_out, S->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
    return MLS2MC_OK;
}


int mls2mc_pcn_step_da(mls2mc_ctx* ctx, const mls2mc_stage* st, int64_t N, double* theta, double* G_lo,
                       double* G_hi, double* phi_lo, double* phi_hi, const double* y, const double* xi,
                       const double* u1, const double* u2, uint8_t* accepted_out, uint8_t* stage1_out,
                       int64_t* n_solved_lo, int64_t* n_solved_hi, void* stream)
{
    MLS_REQUIRE(ctx != nullptr && st != nullptr, "pcn_step_da: null argument");
    MLS_REQUIRE(ctx->sur != nullptr || ctx->d_sur_S != nullptr,
                "pcn_step_da: no surrogate (mls2mc_surrogate_init or mls2mc_set_linear_surrogate)");
    MLS_REQUIRE(st->kernel == MLS2MC_KERNEL_PCN, "pcn_step_da: delayed acceptance is built for the pCN kernel");
    MLS_REQUIRE(st->l_lo >= ctx->prob.l_min && st->l_lo <= ctx->prob.l_max, "pcn_step_da: level outside the context");
    const bool bridge = st->l_hi != st->l_lo;
    if (bridge) {
        MLS_REQUIRE(st->l_hi == st->l_lo + 1 && st->l_hi <= ctx->prob.l_max, "pcn_step_da: bridging needs l_hi = l_lo + 1");
        MLS_REQUIRE(st->zeta >= 0.0 && st->zeta <= 1.0, "pcn_step_da: need 0 <= zeta <= 1");
    }
    MLS_REQUIRE(st->s > 0.0 && st->s <= 1.0 && st->beta >= 0.0 && st->beta <= 1.0, "pcn_step_da: bad s or beta");
    MLS_REQUIRE(N >= 0 && N <= (int64_t(1) << 26), "pcn_step_da: need 0 <= N <= 2^26");
    if (N == 0) return MLS2MC_OK;
    MLS_REQUIRE(theta && y && xi && u1 && u2 && accepted_out, "pcn_step_da: null pointer");
    const bool need_lo = !bridge || st->zeta < 1.0, need_hi = bridge;
    MLS_REQUIRE(!need_lo || (G_lo && phi_lo), "pcn_step_da: null coarse-level cache");
    MLS_REQUIRE(!need_hi || (G_hi && phi_hi), "pcn_step_da: null fine-level cache");
    const hipStream_t s = (hipStream_t)stream;
    const int K = ctx->prob.K, nobs = ctx->nobs;
    // scratch layout (doubles, then ints)
    const size_t nd = (size_t)N * (2 * K + 4 * nobs + 4) + 8;
    const size_t bytes = nd * sizeof(double) + (size_t)N * (sizeof(int32_t) * 3 + 2) + 64;
    MLS_TRY(ctx->ws_da.ensure(bytes));
    double* p = ctx->ws_da.as<double>();
    double* thn = p; p += (size_t)N * K;
    double* thc = p; p += (size_t)N * K;
    double* Gs = p; p += (size_t)N * nobs;       // surrogate outputs (old, then new)
    double* Gcl = p; p += (size_t)N * nobs;
    double* Gch = p; p += (size_t)N * nobs;
    double* Gs2 = p; p += (size_t)N * nobs;
    double* ps_old = p; p += N;
    double* ps_new = p; p += N;
    double* pcl = p; p += N;
    double* pch = p; p += N;
    int64_t* count = reinterpret_cast<int64_t*>(p); p += 8;
    int32_t* idx = reinterpret_cast<int32_t*>(p);
    int32_t* itl = idx + N;
    int32_t* ith = itl + N;
    int8_t* stl = reinterpret_cast<int8_t*>(ith + N);
    int8_t* sth = stl + N;
    const double inv_sigma = 1.0 / ctx->prob.sigma_n;
    MLS_TRY(launch_pcn_propose(N, K, st->s, MLS2MC_KERNEL_PCN, theta, xi, thn, s));
    MLS_TRY(mls2mc_surrogate_predict(ctx, N, theta, Gs, stream));
    MLS_TRY(mls2mc_surrogate_predict(ctx, N, thn, Gs2, stream));
    const unsigned gN = (unsigned)((N + 255) / 256);
    da_psis_kernel<<<gN, 256, 0, s>>>(N, nobs, Gs, y, inv_sigma, st->beta, ps_old);
    da_psis_kernel<<<gN, 256, 0, s>>>(N, nobs, Gs2, y, inv_sigma, st->beta, ps_new);
    da_stage1_kernel<<<1, 1024, 0, s>>>(N, u1, ps_old, ps_new, idx, count, accepted_out, stage1_out,
                                        need_lo ? n_solved_lo : nullptr, need_hi ? n_solved_hi : nullptr);
    gather_count_kernel<<<(unsigned)((N * K + 255) / 256), 256, 0, s>>>(N, K, idx, count, thn, thc);
    MLS_CHECK_HIP(hipGetLastError());
    if (need_lo) MLS_TRY(forward_theta(ctx, st->l_lo, N, thc, Gcl, stl, itl, y, pcl, s, count));
    if (need_hi) MLS_TRY(forward_theta(ctx, st->l_hi, N, thc, Gch, sth, ith, y, pch, s, count));
    if (ctx->da_err) {  // the surrogate's error against the finer level's solve
        da_err_kernel<<<1, 256, 0, s>>>(N, count, idx, nobs, Gs2, need_hi ? Gch : Gcl, inv_sigma, ctx->da_err);
        MLS_CHECK_HIP(hipGetLastError());
    }
    const int mode = !bridge ? 0 : (st->zeta < 1.0 ? 1 : 2);
    da_stage2_kernel<<<gN, 256, 0, s>>>(N, count, idx, K, nobs, mode, st->beta, st->zeta, u2, ps_old, ps_new, thn,
                                       Gcl, Gch, pcl, pch, stl, sth, theta, G_lo, G_hi, phi_lo, phi_hi,
                                       accepted_out);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

}  // extern "C"
