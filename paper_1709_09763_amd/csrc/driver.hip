// The MLS^2MC sampler (Sec. 4) on the device: a host loop that takes the
// per-stage decisions of the update scheme of Sec. 4.4 and enqueues the
// kernels of each stage.  Tempering updates follow Sec. 3.1, level updates
// bridge Phi_l -> Phi_{l+1} at the current inverse temperature through
// adaptive sub-steps (Secs. 3.2, 4.1); every sub-step reweights, resamples
// and moves the particles with pCN (Sec. 2.4).  The first update and every
// update following a level update are tempering updates; otherwise cv^LU is
// estimated on the first J_tilde particles and a level update is taken when
// cv^LU >= tau_LU, reusing those J_tilde solves.  At beta = 1 the remaining
// levels are bridged.
#include <chrono>
#include <cmath>

#include "common.h"

extern "C" int mls2mc_decide(double beta, int l, int l_max, int prev_lu, int scheme, double cv_lu,
                             double tau_lu, double tau_min)
{
    if (l > l_max || !(beta >= 0.0 && beta <= 1.0) ||
        (scheme != MLS2MC_SCHEME_MLS2MC && scheme != MLS2MC_SCHEME_MLB))
        return -1;
    if (beta == 1.0) {
        if (l == l_max) return MLS2MC_DECIDE_DONE;
        if (tau_min > 0.0) {
            if (cv_lu < 0.0) return MLS2MC_DECIDE_NEED_CV;
            if (cv_lu < tau_min) return MLS2MC_DECIDE_DONE;
        }
        return MLS2MC_DECIDE_LU;
    }
    if (scheme == MLS2MC_SCHEME_MLB || l == l_max || prev_lu) return MLS2MC_DECIDE_ITU;
    if (cv_lu < 0.0) return MLS2MC_DECIDE_NEED_CV;
    return cv_lu < tau_lu ? MLS2MC_DECIDE_ITU : MLS2MC_DECIDE_LU;
}

namespace mls {

enum { ST_PRIOR = 0, ST_RESAMPLE = 3, ST_PCN_XI = 4, ST_PCN_U = 5, ST_PCN_U2 = 6 };

__global__ void diff_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                            double* __restrict__ d)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) d[t] = a[t] - b[t];
}

__global__ void zero_kernel(int n, double* __restrict__ v)
{
    if ((int)threadIdx.x < n) v[threadIdx.x] = 0.0;
}

__global__ void count_u8_kernel(int64_t n, const uint8_t* __restrict__ v, int64_t* __restrict__ out)
{
    __shared__ int64_t part[256];
    int64_t s = 0;
    for (int64_t t = threadIdx.x; t < n; t += 256) s += v[t];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t a = 0;
        for (int k = 0; k < 256; ++k) a += part[k];
        out[0] += a;
    }
}

struct RunState {
    double *theta, *Glo, *Ghi, *plo, *phi;      // current state
    double *theta2, *Glo2, *Ghi2, *plo2, *phi2; // gather targets
    double *d, *w, *u, *xi, *upcn, *upcn2, *out3, *cv, *sur_err;
    int32_t* anc;
    uint8_t* acc;
    uint8_t* pass1;
    int64_t* counters;  // [iters, not converged, accepted, -, -, -, -, -, DA solves per level 8..23]
    int8_t* st;
    int32_t* it;
};

}  // namespace mls

using namespace mls;

extern "C" int mls2mc_run(mls2mc_ctx* ctx, const mls2mc_run_config* cfg, const double* y,
                          double* theta_out, mls2mc_run_result* res, void* stream)
{
    MLS_REQUIRE(ctx && cfg && y && theta_out && res, "run: null argument");
    const int64_t J = cfg->J;
    MLS_REQUIRE(J >= 1 && J <= (int64_t(1) << 26), "run: need 1 <= J <= 2^26");
    const int64_t Jt = cfg->J_tilde > 0 ? cfg->J_tilde : (J < 100 ? J : 100);
    MLS_REQUIRE(Jt >= 1 && Jt <= J, "run: need 1 <= J_tilde <= J");
    MLS_REQUIRE(cfg->tau_star > 0 && cfg->n_mcmc >= 0, "run: need tau_star > 0, n_mcmc >= 0");
    MLS_REQUIRE(cfg->kernel == MLS2MC_KERNEL_PCN || cfg->kernel == MLS2MC_KERNEL_RWM, "run: unknown kernel");
    MLS_REQUIRE(cfg->s_pcn > 0 && cfg->s_pcn <= (cfg->kernel == MLS2MC_KERNEL_RWM ? 10.0 : 1.0),
                "run: need 0 < s_pcn <= 1 (pCN) or <= 10 (random walk)");
    MLS_REQUIRE(cfg->scheme == MLS2MC_SCHEME_MLS2MC || cfg->scheme == MLS2MC_SCHEME_MLB, "run: unknown scheme");
    MLS_REQUIRE(cfg->tau_min >= 0.0, "run: need tau_min >= 0");
    const double tau_ess = (double)J / (1.0 + cfg->tau_star * cfg->tau_star);
    const double tau_lu = cfg->tau_lu > 0 ? cfg->tau_lu : cfg->tau_star;
    const double eps = cfg->eps > 0 ? cfg->eps : 1e-6;
    const int max_stages = cfg->max_stages > 0 ? cfg->max_stages : 4000;
    const int K = ctx->prob.K, nobs = ctx->nobs;
    const hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();

    // ---- state buffers
    size_t nd = 2 * ((size_t)J * K + 2 * (size_t)J * nobs + 2 * (size_t)J);  // state + gather
    nd += 3 * (size_t)J + (size_t)J * K + 2 * (size_t)J + 12;                // d w u xi upcn(2) out3 cv sur_err
    size_t bytes = nd * sizeof(double) + (size_t)J * (sizeof(int32_t) * 2 + 3) + 64 * sizeof(int64_t);
    const bool use_sur = cfg->surrogate != 0;
    const int sur_collect = cfg->sur_collect_max_level;
    const int sur_da = cfg->sur_da_min_level;
    const bool sur_linear = use_sur && ctx->d_sur_S != nullptr;  // a given linear surrogate: nothing to train
    if (sur_linear) {
        MLS_REQUIRE(sur_da >= ctx->prob.l_min && sur_da <= ctx->prob.l_max,
                    "run: the linear surrogate needs l_min <= sur_da_min_level <= l_max");
        MLS_REQUIRE(cfg->kernel == MLS2MC_KERNEL_PCN, "run: delayed acceptance is built for the pCN kernel");
    } else if (use_sur) {
        MLS_REQUIRE(sur_da > ctx->prob.l_min && sur_da <= ctx->prob.l_max && sur_collect < sur_da,
                    "run: surrogate needs l_min < sur_da_min_level <= l_max and sur_collect_max_level < sur_da_min_level");
        MLS_REQUIRE(cfg->kernel == MLS2MC_KERNEL_PCN, "run: delayed acceptance is built for the pCN kernel");
    }
    MLS_TRY(ctx->ws_run.ensure(bytes));
    RunState R;
    double* p = ctx->ws_run.as<double>();
    auto take = [&p](size_t n) { double* r = p; p += n; return r; };
    R.theta = take((size_t)J * K); R.Glo = take((size_t)J * nobs); R.Ghi = take((size_t)J * nobs);
    R.plo = take(J); R.phi = take(J);
    R.theta2 = take((size_t)J * K); R.Glo2 = take((size_t)J * nobs); R.Ghi2 = take((size_t)J * nobs);
    R.plo2 = take(J); R.phi2 = take(J);
    R.d = take(J); R.w = take(J); R.u = take(J); R.xi = take((size_t)J * K); R.upcn = take(J);
    R.upcn2 = take(J);
    R.out3 = take(4); R.cv = take(4); R.sur_err = take(4);
    R.counters = reinterpret_cast<int64_t*>(p); p += 32;
    R.it = reinterpret_cast<int32_t*>(p);
    R.anc = R.it + J;
    R.st = reinterpret_cast<int8_t*>(R.anc + J);
    R.acc = reinterpret_cast<uint8_t*>(R.st + J);
    R.pass1 = R.acc + J;
    MLS_CHECK_HIP(hipMemsetAsync(R.counters, 0, 32 * sizeof(int64_t), s));
    zero_kernel<<<1, 64, 0, s>>>(4, R.sur_err);
    MLS_CHECK_HIP(hipGetLastError());

    res->n_stages = 0;
    res->log_Z = 0.0;
    for (int i = 0; i < 16; ++i) res->solves[i] = 0;
    res->accepted = res->proposed = 0;
    res->stage1_passed = res->da_proposed = 0;
    res->sur_train_seconds = 0.0;
    res->sur_final_loss = 0.0;
    res->graphs_launched = 0;
    res->sur_err_mean = res->sur_err_max = 0.0;
    res->sur_err_count = 0;
    double sur_err_sum = 0.0;
    bool sur_ready = sur_linear;
    // the delayed-acceptance steps accumulate the surrogate's error here while the run lasts
    struct ErrSlot {
        mls2mc_ctx* c;
        ~ErrSlot() { c->da_err = nullptr; }
    } err_slot{ctx};
    ctx->da_err = use_sur ? R.sur_err : nullptr;
    if (use_sur && !sur_linear) {
        MLS_TRY(mls2mc_surrogate_init(ctx, cfg->sur_hidden > 0 ? cfg->sur_hidden : 256,
                                      cfg->sur_pairs > 0 ? cfg->sur_pairs : 20480, cfg->seed ^ 0x51u, stream));
    }

    auto fwd = [&](int l, int64_t n, const double* th, double* G, double* ph) -> int {
        if (n == 0) return MLS2MC_OK;
        MLS_TRY(forward_theta(ctx, l, n, th, G, R.st, R.it, y, ph, s));
        MLS_TRY(launch_reduce_i32(n, R.it, R.st, R.counters, s));
        res->solves[l] += n;
        return MLS2MC_OK;
    };
    auto gather_state = [&](bool with_hi) -> int {
        MLS_TRY(launch_gather(J, K, R.anc, J, R.theta, R.theta2, s));
        MLS_TRY(launch_gather(J, nobs, R.anc, J, R.Glo, R.Glo2, s));
        MLS_TRY(launch_gather(J, 1, R.anc, J, R.plo, R.plo2, s));
        std::swap(R.theta, R.theta2); std::swap(R.Glo, R.Glo2); std::swap(R.plo, R.plo2);
        if (with_hi) {
            MLS_TRY(launch_gather(J, nobs, R.anc, J, R.Ghi, R.Ghi2, s));
            MLS_TRY(launch_gather(J, 1, R.anc, J, R.phi, R.phi2, s));
            std::swap(R.Ghi, R.Ghi2); std::swap(R.phi, R.phi2);
        }
        return MLS2MC_OK;
    };
    double acc_host = 0;
    double s_cur = cfg->s_pcn;
    auto adapt = [&](double acc_rate) {  // pCN step adaptation (optional extension)
        if (!cfg->s_adapt) return;
        const double t = s_cur * std::exp(2.0 * (acc_rate - 0.25));
        s_cur = t < 0.005 ? 0.005 : (t > 1.0 ? 1.0 : t);
    };
    auto mutate = [&](int stage, int l, bool bridge, double beta, double zeta) -> int {
        mls2mc_stage st;
        st.l_lo = l;
        st.l_hi = bridge ? l + 1 : l;
        st.beta = beta;
        st.zeta = bridge ? zeta : 1.0;
        st.s = s_cur;
        st.kernel = cfg->kernel;
        const bool da = sur_ready && l >= sur_da;
        for (int m = 0; m < cfg->n_mcmc; ++m) {
            MLS_TRY(launch_philox(cfg->seed, ST_PCN_XI, (uint32_t)stage, (uint32_t)m, J * K, 1, R.xi, s));
            MLS_TRY(launch_philox(cfg->seed, ST_PCN_U, (uint32_t)stage, (uint32_t)m, J, 0, R.upcn, s));
            if (da) {
                MLS_TRY(launch_philox(cfg->seed, ST_PCN_U2, (uint32_t)stage, (uint32_t)m, J, 0, R.upcn2, s));
                MLS_TRY(mls2mc_pcn_step_da(ctx, &st, J, R.theta, R.Glo, R.Ghi, R.plo, R.phi, y, R.xi, R.upcn,
                                           R.upcn2, R.acc, R.pass1, R.counters + 8 + l, R.counters + 8 + l + 1,
                                           stream));
                count_u8_kernel<<<1, 256, 0, s>>>(J, R.acc, R.counters + 2);
                count_u8_kernel<<<1, 256, 0, s>>>(J, R.pass1, R.counters + 3);
                MLS_CHECK_HIP(hipGetLastError());
                res->proposed += J;
                res->da_proposed += J;
                continue;
            }
            MLS_TRY(mls2mc_pcn_step(ctx, &st, J, R.theta, R.Glo, R.Ghi, R.plo, R.phi, y, R.xi, R.upcn,
                                    R.acc, stream));
            if (use_sur && !sur_linear && !bridge && l <= sur_collect) {  // proposals and their solves -> training pairs
                const double* thn = ctx->ws_pcn.as<double>();
                MLS_TRY(mls2mc_surrogate_add_pairs(ctx, J, thn, thn + (size_t)J * K, stream));
            }
            // iteration statistics of the proposals' solves
            const int32_t* itl = ctx->ws_status.as<int32_t>();
            const int8_t* stl = reinterpret_cast<const int8_t*>(itl + 2 * J);
            const bool need_lo = !bridge || zeta < 1.0;
            if (need_lo) {
                MLS_TRY(launch_reduce_i32(J, itl, stl, R.counters, s));
                res->solves[l] += J;
            }
            if (bridge) {
                MLS_TRY(launch_reduce_i32(J, itl + J, stl + J, R.counters, s));
                res->solves[l + 1] += J;
            }
            count_u8_kernel<<<1, 256, 0, s>>>(J, R.acc, R.counters + 2);
            MLS_CHECK_HIP(hipGetLastError());
            res->proposed += J;
        }
        return MLS2MC_OK;
    };
    auto log_stage = [&](int type, int level, double beta, double zeta, double ess) {
        const int k = res->n_stages;
        if (k < res->max_stage_log) {
            if (res->stage_type) res->stage_type[k] = type;
            if (res->stage_level) res->stage_level[k] = level;
            if (res->stage_beta) res->stage_beta[k] = beta;
            if (res->stage_zeta) res->stage_zeta[k] = zeta;
            if (res->stage_ess) res->stage_ess[k] = ess;
        }
        res->n_stages = k + 1;
    };
    auto read3 = [&](double h[3]) -> int {
        MLS_CHECK_HIP(hipMemcpyAsync(h, R.out3, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        MLS_CHECK_HIP(hipStreamSynchronize(s));
        return MLS2MC_OK;
    };
    auto acc_count = [&](double* out) -> int {  // accepted proposals so far
        int64_t c3[3];
        MLS_CHECK_HIP(hipMemcpyAsync(c3, R.counters, sizeof(c3), hipMemcpyDeviceToHost, s));
        MLS_CHECK_HIP(hipStreamSynchronize(s));
        *out = (double)c3[2];
        return MLS2MC_OK;
    };
    // the stage's surrogate error {sum, max, count} -> per-stage log and run totals
    auto log_sur_err = [&](int stage_idx) -> int {
        double e[3] = {0.0, 0.0, 0.0};
        if (use_sur) {
            MLS_CHECK_HIP(hipMemcpyAsync(e, R.sur_err, sizeof(e), hipMemcpyDeviceToHost, s));
            zero_kernel<<<1, 64, 0, s>>>(4, R.sur_err);
            MLS_CHECK_HIP(hipGetLastError());
            MLS_CHECK_HIP(hipStreamSynchronize(s));
        }
        if (stage_idx < res->max_stage_log) {
            if (res->stage_sur_err_mean) res->stage_sur_err_mean[stage_idx] = e[2] > 0 ? e[0] / e[2] : NAN;
            if (res->stage_sur_err_max) res->stage_sur_err_max[stage_idx] = e[2] > 0 ? e[1] : NAN;
        }
        sur_err_sum += e[0];
        res->sur_err_count += (int64_t)e[2];
        if (e[1] > res->sur_err_max) res->sur_err_max = e[1];
        return MLS2MC_OK;
    };

    // ---- prior draw and first evaluation
    MLS_TRY(launch_philox(cfg->seed, ST_PRIOR, 0, 0, J * K, 1, R.theta, s));
    int l = ctx->prob.l_min;
    double beta = 0.0;
    bool prev_lu = true;  // u(-1) = (0,0): the first update is a tempering update
    MLS_TRY(fwd(l, J, R.theta, R.Glo, R.plo));
    int stage = 0;
    int rc = MLS2MC_OK;
    while (true) {
        if (beta == 1.0 && l == ctx->prob.l_max) break;
        if (use_sur && !sur_ready && l >= sur_da && mls2mc_surrogate_n_pairs(ctx) >= 256) {
            const auto ts = std::chrono::steady_clock::now();
            const int epochs = cfg->sur_epochs > 0 ? cfg->sur_epochs : 15;
            std::vector<float> losses(epochs);
            MLS_TRY(mls2mc_surrogate_train(ctx, epochs, cfg->sur_batch > 0 ? cfg->sur_batch : 256,
                                           cfg->sur_lr > 0 ? cfg->sur_lr : 1e-3, cfg->seed ^ 0x7a11u,
                                           losses.data(), stream));
            res->sur_train_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
            res->sur_final_loss = epochs ? losses.back() : 0.0;
            sur_ready = true;
        }
        if (stage >= max_stages) { set_error("run: stage cap reached"); rc = MLS2MC_ESINGULAR; break; }
        bool do_lu, checked = false;
        // cv^LU of a level update at the current beta, from the first J_tilde particles
        auto look_ahead = [&](double* cv) -> int {
            MLS_TRY(fwd(l + 1, Jt, R.theta, R.Ghi, R.phi));
            MLS_TRY(launch_ess_cv(Jt, R.plo, R.phi, beta, R.cv, s));
            double ess;
            MLS_CHECK_HIP(hipMemcpyAsync(&ess, R.cv, sizeof(double), hipMemcpyDeviceToHost, s));
            MLS_CHECK_HIP(hipStreamSynchronize(s));
            const double c2 = (double)Jt / ess - 1.0;
            *cv = std::sqrt(c2 > 0 ? c2 : 0.0);
            return MLS2MC_OK;
        };
        int dec = mls2mc_decide(beta, l, ctx->prob.l_max, prev_lu ? 1 : 0, cfg->scheme, -1.0, tau_lu,
                                cfg->tau_min);
        if (dec == MLS2MC_DECIDE_NEED_CV) {
            double cv;
            MLS_TRY(look_ahead(&cv));
            checked = true;
            dec = mls2mc_decide(beta, l, ctx->prob.l_max, prev_lu ? 1 : 0, cfg->scheme, cv, tau_lu,
                                cfg->tau_min);
        }
        MLS_REQUIRE(dec >= 0 && dec != MLS2MC_DECIDE_NEED_CV, "run: update-scheme decision failed");
        if (dec == MLS2MC_DECIDE_DONE) break;
        do_lu = dec == MLS2MC_DECIDE_LU;
        if (!do_lu) {
            MLS_TRY(launch_next_step(ctx, J, R.plo, 1.0, beta, tau_ess, eps, R.out3, nullptr, R.w, s));
            double h[3];
            MLS_TRY(read3(h));
            if (!std::isfinite(h[0])) { set_error("run: non-finite potential"); rc = MLS2MC_ENOTCONV; break; }
            res->log_Z += h[1];
            MLS_TRY(launch_philox(cfg->seed, ST_RESAMPLE, (uint32_t)stage, 0, J, 0, R.u, s));
            MLS_TRY(launch_resample(ctx, J, R.w, R.u, R.anc, s));
            MLS_TRY(gather_state(false));
            const double a0 = acc_host;
            MLS_TRY(mutate(stage, l, false, h[0], 1.0));
            MLS_TRY(acc_count(&acc_host));
            if (cfg->n_mcmc) adapt((acc_host - a0) / ((double)J * cfg->n_mcmc));
            beta = h[0];
            log_stage(checked ? 1 : 0, l, beta, 0.0, h[2]);
            if (res->stage_acc_rate && stage < res->max_stage_log)
                res->stage_acc_rate[stage] = cfg->n_mcmc ? (acc_host - a0) / ((double)J * cfg->n_mcmc) : 0.0;
            MLS_TRY(log_sur_err(stage));
            ++stage;
            prev_lu = false;
        } else {
            const int64_t j0 = checked ? Jt : 0;
            MLS_TRY(fwd(l + 1, J - j0, R.theta + j0 * K, R.Ghi + j0 * nobs, R.phi + j0));
            double zeta = 0.0;
            bool first = true;
            while (zeta < 1.0) {
                if (stage >= max_stages) { set_error("run: stage cap reached"); rc = MLS2MC_ESINGULAR; break; }
                diff_kernel<<<(unsigned)((J + 255) / 256), 256, 0, s>>>(J, R.phi, R.plo, R.d);
                MLS_CHECK_HIP(hipGetLastError());
                MLS_TRY(launch_next_step(ctx, J, R.d, beta, zeta, tau_ess, eps, R.out3, nullptr, R.w, s));
                double h[3];
                MLS_TRY(read3(h));
                if (!std::isfinite(h[0])) { set_error("run: non-finite potential"); rc = MLS2MC_ENOTCONV; break; }
                res->log_Z += h[1];
                MLS_TRY(launch_philox(cfg->seed, ST_RESAMPLE, (uint32_t)stage, 0, J, 0, R.u, s));
                MLS_TRY(launch_resample(ctx, J, R.w, R.u, R.anc, s));
                MLS_TRY(gather_state(true));
                const double a0 = acc_host;
                MLS_TRY(mutate(stage, l, true, beta, h[0]));
                MLS_TRY(acc_count(&acc_host));
                if (cfg->n_mcmc) adapt((acc_host - a0) / ((double)J * cfg->n_mcmc));
                zeta = h[0];
                log_stage(first ? (checked ? 2 : 3) : 4, l + 1, beta, zeta, h[2]);
                if (res->stage_acc_rate && stage < res->max_stage_log)
                    res->stage_acc_rate[stage] = cfg->n_mcmc ? (acc_host - a0) / ((double)J * cfg->n_mcmc) : 0.0;
                MLS_TRY(log_sur_err(stage));
                first = false;
                ++stage;
            }
            if (rc != MLS2MC_OK) break;
            ++l;
            std::swap(R.Glo, R.Ghi);
            std::swap(R.plo, R.phi);
            prev_lu = true;
        }
    }
    res->final_level = l;
    res->final_beta = beta;
    MLS_CHECK_HIP(hipMemcpyAsync(theta_out, R.theta, sizeof(double) * J * K, hipMemcpyDeviceToDevice, s));
    int64_t c3[32];
    MLS_CHECK_HIP(hipMemcpyAsync(c3, R.counters, sizeof(c3), hipMemcpyDeviceToHost, s));
    MLS_CHECK_HIP(hipStreamSynchronize(s));
    res->iters_total = c3[0];
    res->not_converged = c3[1];
    res->accepted = c3[2];
    res->stage1_passed = c3[3];
    for (int lv = 0; lv <= kMaxLevel && lv < 16; ++lv) res->solves[lv] += c3[8 + lv];  // delayed-acceptance solves
    res->sur_err_mean = res->sur_err_count ? sur_err_sum / (double)res->sur_err_count : 0.0;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}
