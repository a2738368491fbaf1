// Sampler kernels of MLS^2MC: the Gaussian potential (Sec. 2.1), the
// ESS-adaptive step for tempering and bridging (Secs. 3.1, 3.2, 3.4, 4.1),
// multinomial resampling (Sec. 2.4), and the pCN Markov move.
#include <cmath>

#include "common.h"

namespace mls {

// ------------------------------------------------------------ potential --
__global__ void loglik_kernel(int64_t N, int nobs, const double* __restrict__ G,
                              const double* __restrict__ y, double inv_sigma,
                              double* __restrict__ phi)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= N) return;
    double s = 0.0;
    for (int o = 0; o < nobs; ++o) {
        const double r = (y[o] - G[q * nobs + o]) * inv_sigma;
        s += r * r;
    }
    phi[q] = 0.5 * s;
}

int launch_loglik(mls2mc_ctx* ctx, int64_t N, const double* G, const double* y, double* phi,
                  hipStream_t s)
{
    if (N == 0) return MLS2MC_OK;
    loglik_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(N, ctx->nobs, G, y,
                                                             1.0 / ctx->prob.sigma_n, phi);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// ------------------------------------------------------------ next step --
// One workgroup.  lw_j(t) = (-t*scale) d_j; its maximum is attained at
// min_j d_j (the factor is <= 0 and rounding is monotone), so one minimum
// serves every bisection step.  ESS(t) = (sum e^{lw-m})^2 / sum e^{2(lw-m)}.
constexpr int kNS = 1024;

__device__ double ess_eval(int64_t N, const double* __restrict__ d, double dmin, double scale,
                           double t, double* red)
{
    const double a = -t * scale;
    const double m = a * dmin;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t j = threadIdx.x; j < N; j += kNS) {
        const double v = exp(a * d[j] - m);
        s1 += v;
        s2 += v * v;
    }
    s1 = block_sum<kNS>(s1, red);
    s2 = block_sum<kNS>(s2, red);
    return s1 * s1 / s2;
}

__global__ __launch_bounds__(kNS) void next_step_kernel(int64_t N, const double* __restrict__ d,
                                                        double scale, double cur, double tau,
                                                        double eps, double* __restrict__ out3,
                                                        double* __restrict__ logw,
                                                        double* __restrict__ w)
{
    __shared__ double red[kNS / 64];
    double dmin = INFINITY;
    int bad = 0;
    for (int64_t j = threadIdx.x; j < N; j += kNS) {
        const double v = d[j];
        if (!isfinite(v)) bad = 1;
        dmin = fmin(dmin, v);
    }
    dmin = -block_max<kNS>(-dmin, red);
    const double nbad = block_sum<kNS>((double)bad, red);
    if (nbad > 0.0) {
        if (threadIdx.x == 0) out3[0] = out3[1] = out3[2] = NAN;
        return;
    }
    const double tmax = 1.0 - cur;
    const double tmin = eps < tmax ? eps : tmax;
    double t;
    bool at_end = false;
    if (ess_eval(N, d, dmin, scale, tmax, red) >= tau) {
        t = tmax;
        at_end = true;
    } else if (ess_eval(N, d, dmin, scale, tmin, red) <= tau) {
        t = tmin;
        at_end = (tmin == tmax);
    } else {
        double lo = tmin, hi = tmax;
        for (int it = 0; it < 64; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (ess_eval(N, d, dmin, scale, mid, red) >= tau) lo = mid;
            else hi = mid;
        }
        t = lo;
    }
    const double a = -t * scale;
    const double m = a * dmin;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < N; j += kNS) s += exp(a * d[j] - m);
    s = block_sum<kNS>(s, red);
    const double lse = m + log(s);
    for (int64_t j = threadIdx.x; j < N; j += kNS) {
        const double lw = a * d[j];
        if (logw) logw[j] = lw;
        if (w) w[j] = exp(lw - lse);
    }
    const double e = ess_eval(N, d, dmin, scale, t, red);
    if (threadIdx.x == 0) {
        out3[0] = at_end ? 1.0 : cur + t;
        out3[1] = lse - log((double)N);
        out3[2] = e;
    }
}

int launch_next_step(mls2mc_ctx*, int64_t N, const double* d, double scale, double cur, double tau,
                     double eps, double* out3, double* logw, double* w, hipStream_t s)
{
    next_step_kernel<<<1, kNS, 0, s>>>(N, d, scale, cur, tau, eps, out3, logw, w);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// ESS at t = 1 of the weights exp(-scale d), d = dhi - dlo (dlo may be null:
// d = dhi); out[0] = ESS, out[1] = N / ESS - 1 = (cv^LU)^2 of the level-update
// test of Sec. 4.4 (population variance, so ESS = N / (1 + cv^2)).
__global__ __launch_bounds__(kNS) void ess_diff_kernel(int64_t N, const double* __restrict__ dlo,
                                                       const double* __restrict__ dhi,
                                                       double scale, double* __restrict__ out)
{
    __shared__ double red[kNS / 64];
    const double a = -1.0 * scale;
    double mx = -INFINITY;
    int bad = 0;
    for (int64_t j = threadIdx.x; j < N; j += kNS) {
        const double v = dlo ? dhi[j] - dlo[j] : dhi[j];
        if (!isfinite(v)) bad = 1;
        mx = fmax(mx, a * v);
    }
    mx = block_max<kNS>(mx, red);
    const double nbad = block_sum<kNS>((double)bad, red);
    if (nbad > 0.0) {
        if (threadIdx.x == 0) out[0] = out[1] = NAN;
        return;
    }
    double s1 = 0.0, s2 = 0.0;
    for (int64_t j = threadIdx.x; j < N; j += kNS) {
        const double v = exp(a * (dlo ? dhi[j] - dlo[j] : dhi[j]) - mx);
        s1 += v;
        s2 += v * v;
    }
    s1 = block_sum<kNS>(s1, red);
    s2 = block_sum<kNS>(s2, red);
    if (threadIdx.x == 0) {
        const double e = s1 * s1 / s2;
        out[0] = e;
        out[1] = (double)N / e - 1.0;
    }
}

int launch_ess_cv(int64_t N, const double* dlo, const double* dhi, double scale, double* out,
                  hipStream_t s)
{
    ess_diff_kernel<<<1, kNS, 0, s>>>(N, dlo, dhi, scale, out);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// ------------------------------------------------ linear test model --
// G_l(theta) = (A + 2^{-2l} E) theta (A, E: N_obs x K, row-major), with the
// fused potential when y is given: a stand-in forward map for which the
// tempered and bridged posteriors are Gaussian in closed form.  One thread
// per particle; only the first min(N, *N_dev) rows when N_dev is given.
__global__ void linear_forward_kernel(int64_t N, const int64_t* __restrict__ N_dev, int K, int nobs,
                                      double sc, const double* __restrict__ A,
                                      const double* __restrict__ E, const double* __restrict__ th,
                                      double* __restrict__ G, const double* __restrict__ y,
                                      double inv_sigma, double* __restrict__ phi,
                                      int8_t* __restrict__ status, int32_t* __restrict__ iters)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n = N_dev ? (*N_dev < N ? *N_dev : N) : N;
    if (q >= n) return;
    double ph = 0.0;
    for (int o = 0; o < nobs; ++o) {
        double g = 0.0;
        for (int k = 0; k < K; ++k) g += (A[o * K + k] + sc * E[o * K + k]) * th[q * K + k];
        G[q * nobs + o] = g;
        if (y) {
            const double r = (y[o] - g) * inv_sigma;
            ph += r * r;
        }
    }
    if (y && phi) phi[q] = 0.5 * ph;
    if (status) status[q] = 0;
    if (iters) iters[q] = 0;
}

int launch_linear_forward(mls2mc_ctx* ctx, int l, int64_t N, const double* theta, double* G,
                          int8_t* status, int32_t* iters, const double* y, double* phi,
                          hipStream_t s, const int64_t* N_dev)
{
    if (N == 0) return MLS2MC_OK;
    linear_forward_kernel<<<(unsigned)((N + 127) / 128), 128, 0, s>>>(
        N, N_dev, ctx->prob.K, ctx->nobs, std::ldexp(1.0, -2 * l), ctx->d_lin_A, ctx->d_lin_E, theta, G, y,
        1.0 / ctx->prob.sigma_n, phi, status, iters);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// G = S theta for N rows (the linear surrogate; S is N_obs x K)
int launch_linear_map(int64_t N, int K, int nobs, const double* S, const double* theta, double* G, hipStream_t s)
{
    if (N == 0) return MLS2MC_OK;
    linear_forward_kernel<<<(unsigned)((N + 127) / 128), 128, 0, s>>>(N, nullptr, K, nobs, 0.0, S, S, theta, G,
                                                                      nullptr, 0.0, nullptr, nullptr, nullptr);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// ------------------------------------------------------------- resample --
// Exact integer CDF (see mls2mc.h).  One workgroup; thread k owns the
// contiguous chunk [k N / BS, (k+1) N / BS) for the quantised prefix sums.
__global__ __launch_bounds__(kNS) void resample_kernel(int64_t N, const double* __restrict__ w,
                                                       const double* __restrict__ u,
                                                       uint64_t* __restrict__ C,
                                                       int32_t* __restrict__ anc)
{
    __shared__ double red[kNS / 64];
    __shared__ uint64_t part[kNS];
    double mx = 0.0;
    int bad = 0;
    for (int64_t j = threadIdx.x; j < N; j += kNS) {
        const double v = w[j];
        if (!(v >= 0.0) || isinf(v)) bad = 1;
        else mx = fmax(mx, v);
    }
    for (int64_t i = threadIdx.x; i < N; i += kNS) {
        const double v = u[i];
        if (!(v >= 0.0 && v < 1.0)) bad = 1;
    }
    mx = block_max<kNS>(mx, red);
    const double nbad = block_sum<kNS>((double)bad, red);
    if (nbad > 0.0 || !(mx > 0.0)) {
        for (int64_t i = threadIdx.x; i < N; i += kNS) anc[i] = -1;
        return;
    }
    int ex;
    frexp(mx, &ex);
    int c = 0;
    while ((int64_t(1) << c) < N) ++c;
    const int64_t lo = (int64_t)threadIdx.x * N / kNS, hi = (int64_t)(threadIdx.x + 1) * N / kNS;
    uint64_t run = 0;
    for (int64_t j = lo; j < hi; ++j) {
        run += (uint64_t)floor(ldexp(ldexp(w[j], -ex), 62 - c));
        C[j] = run;
    }
    part[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {  // exclusive scan of the chunk totals (exact integers)
        uint64_t acc = 0;
        for (int k = 0; k < kNS; ++k) {
            const uint64_t v = part[k];
            part[k] = acc;
            acc += v;
        }
    }
    __syncthreads();
    const uint64_t off = part[threadIdx.x];
    for (int64_t j = lo; j < hi; ++j) C[j] += off;
    __syncthreads();
    __threadfence_block();
    const uint64_t T = C[N - 1];
    for (int64_t i = threadIdx.x; i < N; i += kNS) {
        const uint64_t U = (uint64_t)ldexp(u[i], 53);
        const uint64_t ph = __umul64hi(U, T), pl = U * T;
        const uint64_t ti = (ph << 11) | (pl >> 53);
        int64_t a = 0, b = N - 1;
        while (a < b) {
            const int64_t mid = a + (b - a) / 2;
            if (C[mid] > ti) b = mid; else a = mid + 1;
        }
        anc[i] = (int32_t)a;
    }
}

// C: N uint64 of scratch for the prefix sums (every entry is written before
// it is read, so it needs no clearing)
int launch_resample_into(int64_t N, const double* w, const double* u, uint64_t* C, int32_t* anc,
                         hipStream_t s)
{
    resample_kernel<<<1, kNS, 0, s>>>(N, w, u, C, anc);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

int launch_resample(mls2mc_ctx* ctx, int64_t N, const double* w, const double* u, int32_t* anc,
                    hipStream_t s)
{
    MLS_TRY(ctx->ws_misc.ensure(sizeof(uint64_t) * (size_t)N));
    return launch_resample_into(N, w, u, ctx->ws_misc.as<uint64_t>(), anc, s);
}

// --------------------------------------------------------------- gather --
__global__ void gather_kernel(int64_t N, int64_t ncols, const int32_t* __restrict__ anc,
                              int64_t n_src, const double* __restrict__ src,
                              double* __restrict__ dst)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * ncols) return;
    const int64_t i = t / ncols, c = t - i * ncols;
    const int64_t a = anc[i];
    dst[t] = (a >= 0 && a < n_src) ? src[a * ncols + c] : NAN;
}

int launch_gather(int64_t N, int64_t ncols, const int32_t* anc, int64_t n_src, const double* src,
                  double* dst, hipStream_t s)
{
    if (N * ncols == 0) return MLS2MC_OK;
    gather_kernel<<<(unsigned)((N * ncols + 255) / 256), 256, 0, s>>>(N, ncols, anc, n_src, src,
                                                                     dst);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// --------------------------------------------------------------- Philox --
// Philox4x32-10 (Salmon et al., SC'11): counter {idx, sub, stage, stream},
// key {seed lo, seed hi}.
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo)
{
    return (double)((((uint64_t)hi << 32) | lo) >> 11) * 0x1.0p-53;
}

__global__ void philox_kernel(uint64_t seed, uint32_t stream_id, uint32_t stage, uint32_t sub,
                              int64_t n, int normal, double* __restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {(uint32_t)i, sub, stage, stream_id};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    if (!normal) {
        out[i] = u53(c[0], c[1]);
    } else {
        const double u1 = 1.0 - u53(c[0], c[1]);
        const double u2 = u53(c[2], c[3]);
        out[i] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
    }
}

int launch_philox(uint64_t seed, uint32_t stream_id, uint32_t stage, uint32_t sub, int64_t n,
                  int normal, double* out, hipStream_t s)
{
    if (n == 0) return MLS2MC_OK;
    philox_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(seed, stream_id, stage, sub, n,
                                                             normal, out);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// ------------------------------------------------------------------ pCN --
__global__ void pcn_propose_kernel(int64_t n, double a, double s, const double* __restrict__ th,
                                   const double* __restrict__ xi, double* __restrict__ out)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) out[t] = a * th[t] + s * xi[t];
}

// pCN: theta' = sqrt(1 - s^2) theta + s xi; random walk: theta' = theta + s xi
int launch_pcn_propose(int64_t N, int K, double s_pcn, int kernel, const double* theta, const double* xi,
                       double* out, hipStream_t s)
{
    const int64_t n = N * K;
    if (n == 0) return MLS2MC_OK;
    const double a = kernel == MLS2MC_KERNEL_RWM ? 1.0 : std::sqrt(1.0 - s_pcn * s_pcn);
    pcn_propose_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, a, s_pcn, theta, xi, out);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// mode 0: tempering (Psi = beta Phi_lo); 1: bridging with zeta < 1; 2:
// bridging at zeta = 1 (Psi = beta Phi_hi).  rwm: the random-walk kernel,
// whose ratio also carries the N(0, I) prior term |theta|^2 / 2.
__global__ void pcn_accept_kernel(int64_t N, int K, int nobs, int mode, int rwm, double beta, double zeta,
                                  const double* __restrict__ u, const double* __restrict__ thn,
                                  const double* __restrict__ Gln, const double* __restrict__ Ghn,
                                  const double* __restrict__ pln, const double* __restrict__ phn,
                                  const int8_t* __restrict__ stl, const int8_t* __restrict__ sth,
                                  double* __restrict__ th, double* __restrict__ Gl,
                                  double* __restrict__ Gh, double* __restrict__ pl,
                                  double* __restrict__ ph, uint8_t* __restrict__ acc)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= N) return;
    const bool need_lo = mode != 2, need_hi = mode != 0;
    double psi_old, psi_new;
    if (mode == 0) {
        psi_old = beta * pl[j];
        psi_new = beta * pln[j];
    } else if (mode == 1) {
        psi_old = beta * ((1.0 - zeta) * pl[j] + zeta * ph[j]);
        psi_new = beta * ((1.0 - zeta) * pln[j] + zeta * phn[j]);
    } else {
        psi_old = beta * ph[j];
        psi_new = beta * phn[j];
    }
    if (rwm) {
        double qo = 0.0, qn = 0.0;
        for (int k = 0; k < K; ++k) {
            qo += th[j * K + k] * th[j * K + k];
            qn += thn[j * K + k] * thn[j * K + k];
        }
        psi_old += 0.5 * qo;
        psi_new += 0.5 * qn;
    }
    bool ok = true;
    if (need_lo && stl && stl[j] != 0) ok = false;
    if (need_hi && sth && sth[j] != 0) ok = false;
    const bool a = ok && (log(u[j]) < -(psi_new - psi_old));
    if (a) {
        for (int k = 0; k < K; ++k) th[j * K + k] = thn[j * K + k];
        if (need_lo) {
            for (int o = 0; o < nobs; ++o) Gl[j * nobs + o] = Gln[j * nobs + o];
            pl[j] = pln[j];
        }
        if (need_hi) {
            for (int o = 0; o < nobs; ++o) Gh[j * nobs + o] = Ghn[j * nobs + o];
            ph[j] = phn[j];
        }
    }
    if (acc) acc[j] = a ? 1 : 0;
}

int launch_pcn_accept(int64_t N, int K, int nobs, int mode, int rwm, double beta, double zeta,
                      const double* u, const double* th_new, const double* Glo_new,
                      const double* Ghi_new, const double* plo_new, const double* phi_new,
                      const int8_t* st_lo, const int8_t* st_hi, double* theta, double* Glo,
                      double* Ghi, double* plo, double* phi, uint8_t* acc, hipStream_t s)
{
    if (N == 0) return MLS2MC_OK;
    pcn_accept_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(
        N, K, nobs, mode, rwm, beta, zeta, u, th_new, Glo_new, Ghi_new, plo_new, phi_new, st_lo, st_hi,
        theta, Glo, Ghi, plo, phi, acc);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

// ---------------------------------------------------- small reductions --
// out2[0] += sum of iters, out2[1] += count of status != 0 (one workgroup).
__global__ __launch_bounds__(kNS) void reduce_iters_kernel(int64_t N, const int32_t* __restrict__ v,
                                                           const int8_t* __restrict__ st,
                                                           int64_t* __restrict__ out2)
{
    __shared__ double red[kNS / 64];
    double a = 0.0, b = 0.0;
    for (int64_t j = threadIdx.x; j < N; j += kNS) {
        a += (double)v[j];
        if (st) b += st[j] != 0 ? 1.0 : 0.0;
    }
    a = block_sum<kNS>(a, red);
    b = block_sum<kNS>(b, red);
    if (threadIdx.x == 0) {
        out2[0] += (int64_t)a;
        out2[1] += (int64_t)b;
    }
}

int launch_reduce_i32(int64_t N, const int32_t* v, const int8_t* st, int64_t* out2, hipStream_t s)
{
    if (N == 0) return MLS2MC_OK;
    reduce_iters_kernel<<<1, kNS, 0, s>>>(N, v, st, out2);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

}  // namespace mls
