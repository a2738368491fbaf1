// extern "C" entry points of libmls2mc (declared in include/mls2mc.h).
#include <cmath>
#include <new>

#include "common.h"

namespace mls {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int DevBuf::ensure(size_t want)
{
    if (want <= bytes) return MLS2MC_OK;
    if (ptr) {
        (void)hipDeviceSynchronize();  // work in flight may still use the old buffer
        hipError_t e = hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
        if (e != hipSuccess) {
            set_error(std::string("hipFree: ") + hipGetErrorString(e));
            return MLS2MC_EDEVICE;
        }
    }
    size_t rounded = (want + (1u << 20) - 1) & ~size_t((1u << 20) - 1);
    if (hipMalloc(&ptr, rounded) != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        set_error("device allocation of " + std::to_string(rounded) + " bytes failed");
        return MLS2MC_ENOMEM;
    }
    bytes = rounded;
    return MLS2MC_OK;
}

void DevBuf::release()
{
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

static int check_level(const mls2mc_ctx* ctx, int l)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(l >= ctx->prob.l_min && l <= ctx->prob.l_max,
                "level " + std::to_string(l) + " outside [l_min, l_max] of the context");
    return MLS2MC_OK;
}

__global__ void chunk_count_kernel(const int64_t* __restrict__ total, int64_t q0, int64_t n,
                                   int64_t* __restrict__ out)
{
    const int64_t r = *total - q0;
    out[0] = r < 0 ? 0 : (r > n ? n : r);
}

// theta -> KL field -> solve, in chunks that bound the field buffer to 2 GiB.
// N_dev (optional, device): only the first min(N, *N_dev) rows are solved.
// The coefficients go through a buffer of at most 8 GiB, so an h = 1/512
// batch runs in launches of 2048 (FP64) or 4096 (mixed) particles: enough
// per launch that the solver's dynamic hand-out of particles evens out
// their differing iteration counts.
constexpr size_t kCoefChunkBytes = 8ull << 30;

int forward_theta(mls2mc_ctx* ctx, int l, int64_t N, const double* theta, double* G,
                  int8_t* status, int32_t* iters, const double* y, double* phi, hipStream_t s,
                  const int64_t* N_dev)
{
    if (ctx->d_lin_A)  // linear test model in place of the PDE
        return launch_linear_forward(ctx, l, N, theta, G, status, iters, y, phi, s, N_dev);
    const bool mixed = ctx->prob.precision == MLS2MC_MIXED;
    const size_t esz = mixed ? sizeof(float) : sizeof(double);
    const int64_t ne = n_elem(l);
    int64_t chunk = (int64_t)(kCoefChunkBytes / (ne * esz));
    if (chunk < 1) chunk = 1;
    if (chunk > N) chunk = N;
    MLS_TRY(ctx->ws_kappa.ensure((size_t)chunk * ne * esz));
    const int K = ctx->prob.K, nobs = ctx->nobs;
    if (N_dev && N > chunk && !ctx->d_chunk_count)
        MLS_CHECK_HIP(hipMalloc(&ctx->d_chunk_count, sizeof(int64_t) * 8));
    for (int64_t q0 = 0; q0 < N; q0 += chunk) {
        const int64_t n = (N - q0 < chunk) ? N - q0 : chunk;
        const int64_t* cnt = N_dev;
        if (N_dev && N > chunk) {
            chunk_count_kernel<<<1, 1, 0, s>>>(N_dev, q0, n, ctx->d_chunk_count);
            MLS_CHECK_HIP(hipGetLastError());
            cnt = ctx->d_chunk_count;
        }
        MLS_TRY(launch_kl_field(ctx, l, n, theta + q0 * K, ctx->ws_kappa.ptr,
                                mixed ? MLS2MC_FIELD_KAPPA_F32 : MLS2MC_FIELD_KAPPA_F64, s, cnt));
        SolveArgs a;
        a.l = l;
        a.N = n;
        a.kappa = ctx->ws_kappa.ptr;
        a.kappa_f32 = mixed;
        a.G = G + q0 * nobs;
        a.status = status ? status + q0 : nullptr;
        a.iters = iters ? iters + q0 : nullptr;
        a.y = y;
        a.phi = phi ? phi + q0 : nullptr;
        a.N_dev = cnt;
        MLS_TRY(launch_solve(ctx, a, s));
    }
    return MLS2MC_OK;
}

int prof_begin(mls2mc_ctx* ctx, int kclass, int l, int64_t items, hipStream_t s, ProfRec* rec)
{
    MLS_CHECK_HIP(hipEventCreate(&rec->a));
    MLS_CHECK_HIP(hipEventCreate(&rec->b));
    MLS_CHECK_HIP(hipEventRecord(rec->a, s));
    ctx->prof[kclass][l].items += items;
    return MLS2MC_OK;
}

int prof_end(mls2mc_ctx* ctx, int kclass, int l, const ProfRec& rec, hipStream_t s)
{
    MLS_CHECK_HIP(hipEventRecord(rec.b, s));
    ctx->prof[kclass][l].recs.push_back(rec);
    return MLS2MC_OK;
}

static void prof_clear(mls2mc_ctx* ctx)
{
    for (auto& row : ctx->prof)
        for (auto& slot : row) {
            for (auto& r : slot.recs) {
                if (r.a) (void)hipEventDestroy(r.a);
                if (r.b) (void)hipEventDestroy(r.b);
            }
            slot.recs.clear();
            slot.items = 0;
        }
}

}  // namespace mls

using namespace mls;

extern "C" {

int mls2mc_profile(mls2mc_ctx* ctx, int enable)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    if (enable) {
        MLS_CHECK_HIP(hipDeviceSynchronize());
        prof_clear(ctx);
        if (!ctx->d_prof_iters)
            MLS_CHECK_HIP(hipMalloc(&ctx->d_prof_iters, sizeof(int64_t) * 2 * (kMaxLevel + 1)));
        MLS_CHECK_HIP(hipMemset(ctx->d_prof_iters, 0, sizeof(int64_t) * 2 * (kMaxLevel + 1)));
    }
    ctx->prof_on = enable != 0;
    return MLS2MC_OK;
}

int mls2mc_profile_read(mls2mc_ctx* ctx, int kclass, int l, mls2mc_prof_entry* out)
{
    MLS_REQUIRE(ctx && out, "profile_read: null argument");
    MLS_REQUIRE(kclass == MLS2MC_PROF_SOLVE || kclass == MLS2MC_PROF_GEMM, "profile_read: bad class");
    MLS_REQUIRE(l >= 0 && l <= kMaxLevel, "profile_read: bad level");
    MLS_CHECK_HIP(hipDeviceSynchronize());
    const ProfSlot& slot = ctx->prof[kclass][l];
    out->launches = (int64_t)slot.recs.size();
    out->items = slot.items;
    out->ms = 0.0;
    for (const auto& r : slot.recs) {
        float ms = 0.f;
        MLS_CHECK_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        out->ms += ms;
    }
    out->iters = 0;
    if (kclass == MLS2MC_PROF_SOLVE && ctx->d_prof_iters) {
        int64_t v[2];
        MLS_CHECK_HIP(hipMemcpy(v, ctx->d_prof_iters + 2 * l, sizeof(v), hipMemcpyDeviceToHost));
        out->iters = v[0];
    }
    return MLS2MC_OK;
}


const char* mls2mc_last_error(void) { return g_last_error.c_str(); }

const char* mls2mc_version(void) { return "mls2mc 1.0 gfx950"; }

int64_t mls2mc_n_elem(int l) { return (l >= 0 && l <= 15) ? n_elem(l) : -1; }
int64_t mls2mc_n_unknowns(int l) { return (l >= 0 && l <= 15) ? n_unk(l) : -1; }
int mls2mc_n_obs(const mls2mc_ctx* ctx) { return ctx ? ctx->nobs : -1; }
int64_t mls2mc_ctx_n_unknowns(const mls2mc_ctx* ctx, int l)
{
    if (!ctx || l < 1 || l > kMaxLevel) return -1;
    return ctx->prob.bc == MLS2MC_BC_FLOW_CELL ? flow_unknowns(l) : n_unk(l);
}

int mls2mc_kl_eigenvalues(const mls2mc_ctx* ctx, double* lambda_out)
{
    MLS_REQUIRE(ctx && lambda_out, "kl_eigenvalues: null argument");
    for (int k = 0; k < ctx->prob.K; ++k) lambda_out[k] = ctx->sqrt_lam[k] * ctx->sqrt_lam[k];
    return MLS2MC_OK;
}

int mls2mc_destroy(mls2mc_ctx* ctx)
{
    if (!ctx) return MLS2MC_OK;
    (void)hipDeviceSynchronize();
    if (ctx->d_modes) (void)hipFree(ctx->d_modes);
    for (int l = 0; l <= kMaxLevel; ++l) {
        if (ctx->d_B[l]) (void)hipFree(ctx->d_B[l]);
        if (ctx->d_B16[l]) (void)hipFree(ctx->d_B16[l]);
        if (ctx->obs[l].idx) (void)hipFree(ctx->obs[l].idx);
        if (ctx->obs[l].w) (void)hipFree(ctx->obs[l].w);
    }
    ctx->ws_solver.release();
    ctx->ws_kappa.release();
    ctx->ws_theta16.release();
    ctx->ws_misc.release();
    ctx->ws_pcn.release();
    ctx->ws_status.release();
    ctx->ws_run.release();
    ctx->ws_prof.release();
    ctx->ws_da.release();
    ctx->ws_list.release();
    ctx->ws_batch.release();
    if (ctx->h_list) (void)hipHostFree(ctx->h_list);
    if (ctx->h_list_ev) (void)hipEventDestroy(ctx->h_list_ev);
    surrogate_destroy(ctx);
    if (ctx->d_chunk_count) (void)hipFree(ctx->d_chunk_count);
    if (ctx->d_queue) (void)hipFree(ctx->d_queue);
    if (ctx->d_lin_A) (void)hipFree(ctx->d_lin_A);
    if (ctx->d_sur_S) (void)hipFree(ctx->d_sur_S);
    prof_clear(ctx);
    if (ctx->d_prof_iters) (void)hipFree(ctx->d_prof_iters);
    delete ctx;
    return MLS2MC_OK;
}

int mls2mc_create(const mls2mc_problem* p, mls2mc_ctx** out)
{
    MLS_REQUIRE(p != nullptr && out != nullptr, "create: null argument");
    *out = nullptr;
    MLS_REQUIRE(p->l_min >= 1 && p->l_max >= p->l_min && p->l_max <= kMaxLevel,
                "create: need 1 <= l_min <= l_max <= 10");
    MLS_REQUIRE(p->K >= 1 && p->K <= 512, "create: need 1 <= K <= 512");
    MLS_REQUIRE(p->sigma2 > 0 && std::isfinite(p->sigma2), "create: sigma2 must be > 0");
    MLS_REQUIRE(p->corr_len > 0 && std::isfinite(p->corr_len), "create: corr_len must be > 0");
    MLS_REQUIRE(p->m >= 1 && p->m <= 32, "create: need 1 <= m <= 32");
    MLS_REQUIRE(p->sigma_n > 0 && std::isfinite(p->sigma_n), "create: sigma_n must be > 0");
    MLS_REQUIRE(p->precision == MLS2MC_FP64 || p->precision == MLS2MC_MIXED,
                "create: unknown precision");
    MLS_REQUIRE(p->rtol >= 0 && p->max_iters >= 0, "create: negative tolerance or cap");
    MLS_REQUIRE(p->cov == MLS2MC_COV_SEPEXP || p->cov == MLS2MC_COV_MATERN32, "create: unknown covariance");
    MLS_REQUIRE(p->cov == MLS2MC_COV_MATERN32 || p->kl_quad == 0,
                "create: kl_quad applies to the Matern covariance only");
    MLS_REQUIRE(p->bc == MLS2MC_BC_DIRICHLET || p->bc == MLS2MC_BC_FLOW_CELL, "create: unknown boundary-value problem");
    MLS_REQUIRE(p->bc == MLS2MC_BC_DIRICHLET || p->precision == MLS2MC_FP64,
                "create: the flow cell is solved in FP64 only (precision)");
    MLS_REQUIRE(p->kl_quad == 0 || (p->kl_quad >= 4 && p->kl_quad <= 128 && p->kl_quad % 2 == 0),
                "create: kl_quad must be even, 4..128");
    MLS_REQUIRE(p->cov != MLS2MC_COV_MATERN32 || p->K <= (p->kl_quad ? p->kl_quad * p->kl_quad : 4096),
                "create: K exceeds the kl_quad^2 Nystrom eigenpairs");
    mls2mc_ctx* ctx = new (std::nothrow) mls2mc_ctx();
    if (!ctx) {
        set_error("create: host allocation failed");
        return MLS2MC_ENOMEM;
    }
    ctx->prob = *p;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        set_error("create: no HIP device");
        return MLS2MC_EDEVICE;
    }
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
            if (prop.multiProcessorCount > 0) ctx->n_cu = prop.multiProcessorCount;
            // leave 1 KiB of the workgroup's LDS to the kernels' static reduction arrays
            if (prop.sharedMemPerBlock > 65536 + 1024) ctx->max_lds = (int)(prop.sharedMemPerBlock - 1024);
        }
    }
    ctx->rtol = p->rtol > 0 ? p->rtol : (p->precision == MLS2MC_MIXED ? 1e-10 : 1e-11);
    ctx->max_iters = p->max_iters > 0 ? p->max_iters : 200;
    int rc = build_kl_tables(ctx);
    if (rc == MLS2MC_OK) rc = build_obs_tables(ctx);
    if (rc == MLS2MC_OK) {  // the solver's work counter starts at zero and resets itself after each launch
        if (hipMalloc(&ctx->d_queue, 2 * sizeof(unsigned long long)) != hipSuccess ||
            hipMemset(ctx->d_queue, 0, 2 * sizeof(unsigned long long)) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess) {
            set_error("create: device allocation failed");
            rc = MLS2MC_ENOMEM;
        }
    }
    if (rc != MLS2MC_OK) {
        std::string msg = g_last_error;
        mls2mc_destroy(ctx);
        g_last_error = msg;
        return rc;
    }
    *out = ctx;
    return MLS2MC_OK;
}

int mls2mc_kl_field(mls2mc_ctx* ctx, int l, int64_t N, const double* theta, void* out, int kind,
                    void* stream)
{
    MLS_TRY(check_level(ctx, l));
    MLS_REQUIRE(N >= 0, "kl_field: N < 0");
    MLS_REQUIRE(N == 0 || (theta && out), "kl_field: null pointer");
    return launch_kl_field(ctx, l, N, theta, out, kind, (hipStream_t)stream);
}

int mls2mc_forward(mls2mc_ctx* ctx, int l, int64_t N, const double* theta, double* G_out,
                   int8_t* status_out, int32_t* iters_out, void* stream)
{
    MLS_TRY(check_level(ctx, l));
    MLS_REQUIRE(N >= 0, "forward: N < 0");
    MLS_REQUIRE(N == 0 || (theta && G_out), "forward: null pointer");
    if (N == 0) return MLS2MC_OK;
    return forward_theta(ctx, l, N, theta, G_out, status_out, iters_out, nullptr, nullptr,
                         (hipStream_t)stream);
}

int mls2mc_forward_field(mls2mc_ctx* ctx, int l, int64_t N, const double* kappa, double* G_out,
                         double* p_out, int8_t* status_out, int32_t* iters_out, void* stream)
{
    MLS_TRY(check_level(ctx, l));
    MLS_REQUIRE(N >= 0, "forward_field: N < 0");
    MLS_REQUIRE(N == 0 || (kappa && G_out), "forward_field: null pointer");
    MLS_REQUIRE(!ctx->d_lin_A, "forward_field: not defined while the linear test model is set");
    if (N == 0) return MLS2MC_OK;
    const hipStream_t s = (hipStream_t)stream;
    const bool mixed = ctx->prob.precision == MLS2MC_MIXED;
    const void* kin = kappa;
    if (mixed) {  // the mixed solver takes FP32 coefficients: round once
        const int64_t n = N * n_elem(l);
        MLS_TRY(ctx->ws_kappa.ensure(sizeof(float) * (size_t)n));
        MLS_TRY(launch_d2f(kappa, ctx->ws_kappa.as<float>(), n, s));
        kin = ctx->ws_kappa.ptr;
    }
    SolveArgs a;
    a.l = l;
    a.N = N;
    a.kappa = kin;
    a.kappa_f32 = mixed;
    a.G = G_out;
    a.p_out = p_out;
    a.status = status_out;
    a.iters = iters_out;
    return launch_solve(ctx, a, s);
}

int mls2mc_loglik(mls2mc_ctx* ctx, int64_t N, const double* G, const double* y, double* phi_out,
                  void* stream)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(N >= 0, "loglik: N < 0");
    MLS_REQUIRE(N == 0 || (G && y && phi_out), "loglik: null pointer");
    return launch_loglik(ctx, N, G, y, phi_out, (hipStream_t)stream);
}

int mls2mc_next_step(mls2mc_ctx* ctx, int64_t N, const double* d, double scale, double cur,
                     double tau_ess, double eps, double* out3, double* logw_out, double* w_out,
                     void* stream)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(N >= 1 && N <= (int64_t(1) << 26), "next_step: need 1 <= N <= 2^26");
    MLS_REQUIRE(d && out3, "next_step: null pointer");
    MLS_REQUIRE(cur >= 0.0 && cur < 1.0, "next_step: need 0 <= cur < 1");
    MLS_REQUIRE(eps > 0.0 && std::isfinite(scale) && scale >= 0.0, "next_step: need eps > 0, scale >= 0");
    return launch_next_step(ctx, N, d, scale, cur, tau_ess, eps, out3, logw_out, w_out,
                            (hipStream_t)stream);
}

int mls2mc_cv_lu(mls2mc_ctx* ctx, int64_t N, const double* d, double scale, double* out2, void* stream)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(N >= 1 && N <= (int64_t(1) << 26), "cv_lu: need 1 <= N <= 2^26");
    MLS_REQUIRE(d && out2, "cv_lu: null pointer");
    MLS_REQUIRE(std::isfinite(scale) && scale >= 0.0, "cv_lu: need scale >= 0");
    return launch_ess_cv(N, nullptr, d, scale, out2, (hipStream_t)stream);
}

int mls2mc_set_linear_model(mls2mc_ctx* ctx, const double* A, const double* E)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE((A == nullptr) == (E == nullptr), "set_linear_model: give both A and E, or neither");
    MLS_CHECK_HIP(hipDeviceSynchronize());  // work in flight may still read the old tables
    if (ctx->d_lin_A) (void)hipFree(ctx->d_lin_A);
    ctx->d_lin_A = ctx->d_lin_E = nullptr;
    if (!A) return MLS2MC_OK;
    const size_t n = (size_t)ctx->nobs * ctx->prob.K;
    for (size_t i = 0; i < n; ++i)
        MLS_REQUIRE(std::isfinite(A[i]) && std::isfinite(E[i]), "set_linear_model: non-finite entry");
    double* d = nullptr;
    if (hipMalloc(&d, 2 * n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("set_linear_model: device allocation failed");
        return MLS2MC_ENOMEM;
    }
    int rc = MLS2MC_OK;
    if (hipMemcpy(d, A, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d + n, E, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(d);
        set_error("set_linear_model: copy to the device failed");
        rc = MLS2MC_EDEVICE;
    } else {
        ctx->d_lin_A = d;
        ctx->d_lin_E = d + n;
    }
    return rc;
}

int mls2mc_set_linear_surrogate(mls2mc_ctx* ctx, const double* S)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_CHECK_HIP(hipDeviceSynchronize());  // work in flight may still read the old table
    if (ctx->d_sur_S) (void)hipFree(ctx->d_sur_S);
    ctx->d_sur_S = nullptr;
    if (!S) return MLS2MC_OK;
    const size_t n = (size_t)ctx->nobs * ctx->prob.K;
    for (size_t i = 0; i < n; ++i) MLS_REQUIRE(std::isfinite(S[i]), "set_linear_surrogate: non-finite entry");
    double* d = nullptr;
    if (hipMalloc(&d, n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("set_linear_surrogate: device allocation failed");
        return MLS2MC_ENOMEM;
    }
    if (hipMemcpy(d, S, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(d);
        set_error("set_linear_surrogate: copy to the device failed");
        return MLS2MC_EDEVICE;
    }
    ctx->d_sur_S = d;
    return MLS2MC_OK;
}

int mls2mc_resample(mls2mc_ctx* ctx, int64_t N, const double* w, const double* u, int32_t* anc_out,
                    void* stream)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(N >= 1 && N <= (int64_t(1) << 26), "resample: need 1 <= N <= 2^26");
    MLS_REQUIRE(w && u && anc_out, "resample: null pointer");
    return launch_resample(ctx, N, w, u, anc_out, (hipStream_t)stream);
}

int mls2mc_gather(mls2mc_ctx* ctx, int64_t N, int64_t ncols, const int32_t* anc, int64_t n_src,
                  const double* src, double* dst, void* stream)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(N >= 0 && ncols >= 0 && n_src >= 0, "gather: negative size");
    MLS_REQUIRE(N * ncols == 0 || (anc && src && dst), "gather: null pointer");
    MLS_REQUIRE(src != dst, "gather: src and dst must differ");
    return launch_gather(N, ncols, anc, n_src, src, dst, (hipStream_t)stream);
}

int mls2mc_philox_fill(mls2mc_ctx* ctx, uint64_t seed, uint32_t stream_id, uint32_t stage,
                       uint32_t sub, int64_t n, int normal, double* out, void* stream)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(n >= 0 && n <= (int64_t(1) << 32), "philox_fill: need 0 <= n <= 2^32");
    MLS_REQUIRE(n == 0 || out, "philox_fill: null pointer");
    return launch_philox(seed, stream_id, stage, sub, n, normal, out, (hipStream_t)stream);
}

int mls2mc_pcn_step(mls2mc_ctx* ctx, const mls2mc_stage* st, int64_t N, double* theta,
                    double* G_lo, double* G_hi, double* phi_lo, double* phi_hi, const double* y,
                    const double* xi, const double* u, uint8_t* accepted_out, void* stream)
{
    MLS_REQUIRE(ctx != nullptr && st != nullptr, "pcn_step: null argument");
    MLS_TRY(check_level(ctx, st->l_lo));
    const bool bridge = st->l_hi != st->l_lo;
    if (bridge) {
        MLS_REQUIRE(st->l_hi == st->l_lo + 1, "pcn_step: bridging needs l_hi = l_lo + 1");
        MLS_TRY(check_level(ctx, st->l_hi));
        MLS_REQUIRE(st->zeta >= 0.0 && st->zeta <= 1.0, "pcn_step: need 0 <= zeta <= 1");
    }
    MLS_REQUIRE(st->kernel == MLS2MC_KERNEL_PCN || st->kernel == MLS2MC_KERNEL_RWM,
                "pcn_step: kernel must be MLS2MC_KERNEL_PCN or MLS2MC_KERNEL_RWM");
    MLS_REQUIRE(st->s > 0.0 && st->s <= (st->kernel == MLS2MC_KERNEL_RWM ? 10.0 : 1.0),
                "pcn_step: need 0 < s <= 1 (pCN) or 0 < s <= 10 (random walk)");
    MLS_REQUIRE(st->beta >= 0.0 && st->beta <= 1.0, "pcn_step: need 0 <= beta <= 1");
    MLS_REQUIRE(N >= 0, "pcn_step: N < 0");
    if (N == 0) return MLS2MC_OK;
    MLS_REQUIRE(theta && y && xi && u, "pcn_step: null pointer");
    const bool need_lo = !bridge || st->zeta < 1.0;
    const bool need_hi = bridge;
    MLS_REQUIRE(!need_lo || (G_lo && phi_lo), "pcn_step: null coarse-level cache");
    MLS_REQUIRE(!need_hi || (G_hi && phi_hi), "pcn_step: null fine-level cache");
    const hipStream_t s = (hipStream_t)stream;
    const int K = ctx->prob.K, nobs = ctx->nobs;
    // scratch: theta' (N K), G' lo/hi (N nobs each), phi' lo/hi (N each)
    const size_t nd = (size_t)N * K + 2 * (size_t)N * nobs + 2 * (size_t)N;
    MLS_TRY(ctx->ws_pcn.ensure(sizeof(double) * nd));
    double* thn = ctx->ws_pcn.as<double>();
    double* Gln = thn + (size_t)N * K;
    double* Ghn = Gln + (size_t)N * nobs;
    double* pln = Ghn + (size_t)N * nobs;
    double* phn = pln + N;
    MLS_TRY(ctx->ws_status.ensure((size_t)N * 2 * (sizeof(int8_t) + sizeof(int32_t)) + 64));
    int32_t* itl = ctx->ws_status.as<int32_t>();
    int32_t* ith = itl + N;
    int8_t* stl = reinterpret_cast<int8_t*>(ith + N);
    int8_t* sth = stl + N;
    MLS_TRY(launch_pcn_propose(N, K, st->s, st->kernel, theta, xi, thn, s));
    if (need_lo) MLS_TRY(forward_theta(ctx, st->l_lo, N, thn, Gln, stl, itl, y, pln, s));
    if (need_hi) MLS_TRY(forward_theta(ctx, st->l_hi, N, thn, Ghn, sth, ith, y, phn, s));
    const int mode = !bridge ? 0 : (st->zeta < 1.0 ? 1 : 2);
    return launch_pcn_accept(N, K, nobs, mode, st->kernel == MLS2MC_KERNEL_RWM, st->beta, st->zeta, u, thn,
                             Gln, Ghn, pln, phn,
                             need_lo ? stl : nullptr, need_hi ? sth : nullptr, theta, G_lo, G_hi,
                             phi_lo, phi_hi, accepted_out, s);
}

}  // extern "C"

// ------------------------------------------------------------ helpers --
namespace mls {

__global__ void d2f_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) b[t] = (float)a[t];
}

int launch_d2f(const double* a, float* b, int64_t n, hipStream_t s)
{
    if (n == 0) return MLS2MC_OK;
    d2f_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, b, n);
    MLS_CHECK_HIP(hipGetLastError());
    return MLS2MC_OK;
}

}  // namespace mls
