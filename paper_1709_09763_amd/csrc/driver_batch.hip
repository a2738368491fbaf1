// Many independent MLS^2MC instances (Sec. 4, update scheme of Sec. 4.4) in
// lock-step rounds.  In every round each active instance performs one SMC
// sub-step (a tempering update or one bridging sub-step): reweight, resample
// and n_mcmc pCN moves.  All forward solves of a phase, across instances and
// levels, go into one fused work-list launch, and the mutation phase of the
// round is captured as a HIP graph and launched once.  Each instance draws
// the same Philox streams as mls2mc_run with its seed, so it reproduces the
// single-instance run.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "common.h"

namespace mls {

namespace {

enum { ST_PRIOR = 0, ST_RESAMPLE = 3, ST_PCN_XI = 4, ST_PCN_U = 5 };

__global__ void diff_kernel_b(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                              double* __restrict__ d)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) d[t] = a[t] - b[t];
}

__global__ void count_acc_kernel(int64_t n, const uint8_t* __restrict__ v, int64_t* __restrict__ out)
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

struct Inst {
    int64_t J, Jt;
    int lmax;
    const double* y;
    uint64_t seed;
    double* out;
    // host state
    int l = 0;
    double beta = 0.0, zeta = 0.0, t_next = 0.0;
    bool prev_lu = true, in_lu = false, lu_first = false, checked = false, done = false;
    int stage = 0;
    // device state
    double *theta, *Glo, *Ghi, *plo, *phi, *theta2, *Glo2, *Ghi2, *plo2, *phi2;
    double *thn, *Gnl, *Gnh, *pnl, *pnh, *d, *w, *u, *xi, *upcn, *out3, *cv;
    int32_t *itl, *ith, *anc;
    int8_t *stl, *sth;
    uint8_t* acc;
    int64_t* counters;  // [accepted]
};

size_t inst_bytes(int64_t J, int K, int nobs)
{
    const size_t nd = 2 * ((size_t)J * K + 2 * (size_t)J * nobs + 2 * (size_t)J)   // state + gather
                      + (size_t)J * K + 2 * (size_t)J * nobs + 2 * (size_t)J        // proposals
                      + 3 * (size_t)J + (size_t)J * K + (size_t)J + 8;              // d w u xi upcn out3 cv
    return ((nd * sizeof(double) + (size_t)J * (3 * sizeof(int32_t) + 3) + 8 * sizeof(int64_t)) + 255) & ~size_t(255);
}

void inst_carve(Inst& I, char* base, int K, int nobs)
{
    double* p = (double*)base;
    auto take = [&p](size_t n) { double* r = p; p += n; return r; };
    const int64_t J = I.J;
    I.theta = take((size_t)J * K); I.Glo = take((size_t)J * nobs); I.Ghi = take((size_t)J * nobs);
    I.plo = take(J); I.phi = take(J);
    I.theta2 = take((size_t)J * K); I.Glo2 = take((size_t)J * nobs); I.Ghi2 = take((size_t)J * nobs);
    I.plo2 = take(J); I.phi2 = take(J);
    I.thn = take((size_t)J * K); I.Gnl = take((size_t)J * nobs); I.Gnh = take((size_t)J * nobs);
    I.pnl = take(J); I.pnh = take(J);
    I.d = take(J); I.w = take(J); I.u = take(J); I.xi = take((size_t)J * K); I.upcn = take(J);
    I.out3 = take(4); I.cv = take(4);
    I.counters = (int64_t*)p; p += 8;
    I.itl = (int32_t*)p; I.ith = I.itl + J; I.anc = I.ith + J;
    I.stl = (int8_t*)(I.anc + J); I.sth = I.stl + J;
    I.acc = (uint8_t*)(I.sth + J);
}

void log_stage(mls2mc_run_result& r, int type, int level, double beta, double zeta, double ess)
{
    const int k = r.n_stages;
    if (k < r.max_stage_log) {
        if (r.stage_type) r.stage_type[k] = type;
        if (r.stage_level) r.stage_level[k] = level;
        if (r.stage_beta) r.stage_beta[k] = beta;
        if (r.stage_zeta) r.stage_zeta[k] = zeta;
        if (r.stage_ess) r.stage_ess[k] = ess;
    }
    r.n_stages = k + 1;
}

}  // namespace
}  // namespace mls

using namespace mls;

extern "C" int mls2mc_run_batch(mls2mc_ctx* ctx, const mls2mc_run_config* cfg, int n_inst,
                                const mls2mc_instance* inst, mls2mc_run_result* res, int use_graphs,
                                void* stream)
{
    MLS_REQUIRE(ctx && cfg && inst && res, "run_batch: null argument");
    MLS_REQUIRE(n_inst >= 1 && n_inst <= 4096, "run_batch: need 1 <= n_inst <= 4096");
    MLS_REQUIRE(ctx->prob.bc == MLS2MC_BC_DIRICHLET, "run_batch: Dirichlet problem only");
    MLS_REQUIRE(!ctx->d_lin_A, "run_batch: the linear test model runs through the single-instance entry points");
    MLS_REQUIRE(cfg->surrogate == 0 && cfg->s_adapt == 0 && cfg->scheme == MLS2MC_SCHEME_MLS2MC &&
                    cfg->tau_min == 0.0 && cfg->kernel == MLS2MC_KERNEL_PCN,
                "run_batch: the surrogate form, pCN step adaptation, other schemes and kernels, and the "
                "adaptive maximum level run through mls2mc_run");
    MLS_REQUIRE(cfg->tau_star > 0 && cfg->n_mcmc >= 0 && cfg->s_pcn > 0 && cfg->s_pcn <= 1,
                "run_batch: need tau_star > 0, n_mcmc >= 0, 0 < s_pcn <= 1");
    const int K = ctx->prob.K, nobs = ctx->nobs;
    const double eps = cfg->eps > 0 ? cfg->eps : 1e-6;
    const int max_stages = cfg->max_stages > 0 ? cfg->max_stages : 4000;
    const auto t0 = std::chrono::steady_clock::now();
    // a non-default stream: the legacy stream cannot be captured
    hipStream_t s = (hipStream_t)stream;
    hipStream_t own = nullptr;
    if (!s) {
        MLS_CHECK_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        s = own;
    }
    struct StreamGuard {
        hipStream_t h;
        ~StreamGuard() { if (h) { (void)hipStreamSynchronize(h); (void)hipStreamDestroy(h); } }
    } guard{own};

    std::vector<Inst> I(n_inst);
    size_t total = 0;
    for (int i = 0; i < n_inst; ++i) {
        const mls2mc_instance& q = inst[i];
        MLS_REQUIRE(q.J >= 1 && q.J <= (int64_t(1) << 24), "run_batch: need 1 <= J <= 2^24 per instance");
        MLS_REQUIRE(q.l_max >= ctx->prob.l_min && q.l_max <= ctx->prob.l_max, "run_batch: instance l_max outside the context");
        MLS_REQUIRE(q.y && q.theta_out, "run_batch: null instance pointer");
        I[i].J = q.J;
        I[i].Jt = cfg->J_tilde > 0 ? std::min<int64_t>(cfg->J_tilde, q.J) : std::min<int64_t>(100, q.J);
        I[i].lmax = q.l_max;
        I[i].y = q.y;
        I[i].seed = q.seed;
        I[i].out = q.theta_out;
        I[i].l = ctx->prob.l_min;
        total += inst_bytes(q.J, K, nobs);
        mls2mc_run_result& r = res[i];
        r.n_stages = 0; r.log_Z = 0.0; r.accepted = r.proposed = 0; r.iters_total = 0; r.not_converged = 0;
        r.stage1_passed = r.da_proposed = 0; r.sur_train_seconds = 0; r.sur_final_loss = 0;
        r.graphs_launched = 0;
        r.sur_err_mean = r.sur_err_max = 0.0;
        r.sur_err_count = 0;
        for (int k = 0; k < 16; ++k) r.solves[k] = 0;
    }
    MLS_TRY(ctx->ws_batch.ensure(total));
    {
        char* b = (char*)ctx->ws_batch.ptr;
        for (int i = 0; i < n_inst; ++i) {
            inst_carve(I[i], b, K, nobs);
            b += inst_bytes(I[i].J, K, nobs);
        }
    }
    double* hbuf = nullptr;  // pinned: per instance out3 (3) + cv (1) + accepted (1)
    MLS_CHECK_HIP(hipHostMalloc(&hbuf, sizeof(double) * 8 * n_inst));
    struct HostGuard { double* p; ~HostGuard() { if (p) (void)hipHostFree(p); } } hg{hbuf};

    // prior draws and the first evaluation of every instance, one fused launch
    std::vector<FwdItem> items;
    for (auto& q : I) {
        MLS_CHECK_HIP(hipMemsetAsync(q.counters, 0, 8 * sizeof(int64_t), s));
        MLS_TRY(launch_philox(q.seed, ST_PRIOR, 0, 0, q.J * K, 1, q.theta, s));
        items.push_back({q.l, q.J, q.theta, q.Glo, q.y, q.plo, q.stl, q.itl});
    }
    MLS_TRY(forward_list(ctx, items, s));
    for (int i = 0; i < n_inst; ++i) res[i].solves[I[i].l] += I[i].J;
    int64_t graphs = 0;
    int rc = MLS2MC_OK;
    while (rc == MLS2MC_OK) {
        // ---- A: decisions (look-ahead solves fused across instances)
        std::vector<int> check, start_lu;
        for (int i = 0; i < n_inst; ++i) {
            Inst& q = I[i];
            if (q.done || q.in_lu) continue;
            if (q.beta == 1.0 && q.l == q.lmax) { q.done = true; continue; }
            if (q.stage >= max_stages) { set_error("run_batch: stage cap reached"); rc = MLS2MC_ESINGULAR; break; }
            q.checked = false;
            if (q.beta == 1.0) start_lu.push_back(i);
            else if (q.l == q.lmax || q.prev_lu) continue;  // tempering
            else check.push_back(i);
        }
        if (rc != MLS2MC_OK) break;
        if (!check.empty()) {
            items.clear();
            for (int i : check) items.push_back({I[i].l + 1, I[i].Jt, I[i].theta, I[i].Ghi, I[i].y, I[i].phi, I[i].sth, I[i].ith});
            MLS_TRY(forward_list(ctx, items, s));
            for (int i : check) {
                res[i].solves[I[i].l + 1] += I[i].Jt;
                MLS_TRY(launch_ess_cv(I[i].Jt, I[i].plo, I[i].phi, I[i].beta, I[i].cv, s));
                MLS_CHECK_HIP(hipMemcpyAsync(hbuf + 8 * i + 3, I[i].cv, sizeof(double), hipMemcpyDeviceToHost, s));
            }
            MLS_CHECK_HIP(hipStreamSynchronize(s));
            const double tau_lu = cfg->tau_lu > 0 ? cfg->tau_lu : cfg->tau_star;
            for (int i : check) {
                const double c2 = (double)I[i].Jt / hbuf[8 * i + 3] - 1.0;
                const double cv = std::sqrt(c2 > 0 ? c2 : 0.0);
                I[i].checked = true;
                if (!(cv < tau_lu)) start_lu.push_back(i);
            }
        }
        if (!start_lu.empty()) {
            items.clear();
            for (int i : start_lu) {
                Inst& q = I[i];
                const int64_t j0 = q.checked ? q.Jt : 0;
                if (q.J - j0 > 0)
                    items.push_back({q.l + 1, q.J - j0, q.theta + j0 * K, q.Ghi + j0 * nobs, q.y, q.phi + j0, q.sth, q.ith});
                res[i].solves[q.l + 1] += q.J - j0;
                q.in_lu = true;
                q.lu_first = true;
                q.zeta = 0.0;
            }
            MLS_TRY(forward_list(ctx, items, s));
        }
        std::vector<int> act;
        for (int i = 0; i < n_inst; ++i)
            if (!I[i].done) act.push_back(i);
        if (act.empty()) break;
        // ---- B: adaptive next temperature / bridging parameter
        for (int i : act) {
            Inst& q = I[i];
            const double tau = (double)q.J / (1.0 + cfg->tau_star * cfg->tau_star);
            if (q.in_lu) {
                diff_kernel_b<<<(unsigned)((q.J + 255) / 256), 256, 0, s>>>(q.J, q.phi, q.plo, q.d);
                MLS_CHECK_HIP(hipGetLastError());
                MLS_TRY(launch_next_step(ctx, q.J, q.d, q.beta, q.zeta, tau, eps, q.out3, nullptr, q.w, s));
            } else {
                MLS_TRY(launch_next_step(ctx, q.J, q.plo, 1.0, q.beta, tau, eps, q.out3, nullptr, q.w, s));
            }
            MLS_CHECK_HIP(hipMemcpyAsync(hbuf + 8 * i, q.out3, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        MLS_CHECK_HIP(hipStreamSynchronize(s));
        for (int i : act) {
            if (!std::isfinite(hbuf[8 * i])) { set_error("run_batch: non-finite potential"); rc = MLS2MC_ENOTCONV; }
            I[i].t_next = hbuf[8 * i];
            res[i].log_Z += hbuf[8 * i + 1];
        }
        if (rc != MLS2MC_OK) break;
        // ---- C: resample and gather
        for (int i : act) {
            Inst& q = I[i];
            MLS_TRY(launch_philox(q.seed, ST_RESAMPLE, (uint32_t)q.stage, 0, q.J, 0, q.u, s));
            MLS_TRY(launch_resample(ctx, q.J, q.w, q.u, q.anc, s));
            MLS_TRY(launch_gather(q.J, K, q.anc, q.J, q.theta, q.theta2, s));
            MLS_TRY(launch_gather(q.J, nobs, q.anc, q.J, q.Glo, q.Glo2, s));
            MLS_TRY(launch_gather(q.J, 1, q.anc, q.J, q.plo, q.plo2, s));
            std::swap(q.theta, q.theta2); std::swap(q.Glo, q.Glo2); std::swap(q.plo, q.plo2);
            if (q.in_lu) {
                MLS_TRY(launch_gather(q.J, nobs, q.anc, q.J, q.Ghi, q.Ghi2, s));
                MLS_TRY(launch_gather(q.J, 1, q.anc, q.J, q.phi, q.phi2, s));
                std::swap(q.Ghi, q.Ghi2); std::swap(q.phi, q.phi2);
            }
        }
        // ---- D: mutation, one fused forward per pCN step, captured as a graph
        items.clear();
        for (int i : act) {
            Inst& q = I[i];
            const bool need_lo = !q.in_lu || q.t_next < 1.0;
            if (need_lo) items.push_back({q.l, q.J, q.thn, q.Gnl, q.y, q.pnl, q.stl, q.itl});
            if (q.in_lu) items.push_back({q.l + 1, q.J, q.thn, q.Gnh, q.y, q.pnh, q.sth, q.ith});
        }
        std::vector<ListChunk> chunks;
        MLS_TRY(prepare_list(ctx, items, chunks, s));  // uploads lists, sizes workspaces
        const bool prof = ctx->prof_on;
        ctx->prof_on = false;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        if (use_graphs) MLS_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int erc = MLS2MC_OK;
        for (int m = 0; m < cfg->n_mcmc && erc == MLS2MC_OK; ++m) {
            for (int i : act) {
                Inst& q = I[i];
                if (erc == MLS2MC_OK) erc = launch_philox(q.seed, ST_PCN_XI, (uint32_t)q.stage, (uint32_t)m, q.J * K, 1, q.xi, s);
                if (erc == MLS2MC_OK) erc = launch_philox(q.seed, ST_PCN_U, (uint32_t)q.stage, (uint32_t)m, q.J, 0, q.upcn, s);
                if (erc == MLS2MC_OK) erc = launch_pcn_propose(q.J, K, cfg->s_pcn, MLS2MC_KERNEL_PCN, q.theta, q.xi, q.thn, s);
            }
            if (erc == MLS2MC_OK) erc = enqueue_list(ctx, chunks, s);
            for (int i : act) {
                Inst& q = I[i];
                const int mode = !q.in_lu ? 0 : (q.t_next < 1.0 ? 1 : 2);
                const double beta = q.in_lu ? q.beta : q.t_next;
                if (erc == MLS2MC_OK)
                    erc = launch_pcn_accept(q.J, K, nobs, mode, 0, beta, q.t_next, q.upcn, q.thn, q.Gnl, q.Gnh, q.pnl,
                                            q.pnh, mode != 2 ? q.stl : nullptr, mode != 0 ? q.sth : nullptr, q.theta,
                                            q.Glo, q.Ghi, q.plo, q.phi, q.acc, s);
                if (erc == MLS2MC_OK) {
                    count_acc_kernel<<<1, 256, 0, s>>>(q.J, q.acc, q.counters);
                    if (hipGetLastError() != hipSuccess) erc = MLS2MC_EDEVICE;
                }
            }
        }
        if (use_graphs) {
            hipError_t e = hipStreamEndCapture(s, &graph);
            if (erc == MLS2MC_OK && e != hipSuccess) {
                set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
                erc = MLS2MC_EDEVICE;
            }
            if (erc == MLS2MC_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                set_error("hipGraphInstantiate failed");
                erc = MLS2MC_EDEVICE;
            }
            if (erc == MLS2MC_OK && hipGraphLaunch(exec, s) != hipSuccess) {
                set_error("hipGraphLaunch failed");
                erc = MLS2MC_EDEVICE;
            }
            if (erc == MLS2MC_OK) ++graphs;
        }
        ctx->prof_on = prof;
        if (erc == MLS2MC_OK && exec) erc = hipStreamSynchronize(s) == hipSuccess ? MLS2MC_OK : MLS2MC_EDEVICE;
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        MLS_TRY(erc);
        // ---- E: bookkeeping
        for (int i : act) {
            Inst& q = I[i];
            mls2mc_run_result& r = res[i];
            r.proposed += q.J * cfg->n_mcmc;
            if (q.in_lu) {
                const bool need_lo = q.t_next < 1.0;
                r.solves[q.l + 1] += q.J * cfg->n_mcmc;
                if (need_lo) r.solves[q.l] += q.J * cfg->n_mcmc;
                q.zeta = q.t_next;
                log_stage(r, q.lu_first ? (q.checked ? 2 : 3) : 4, q.l + 1, q.beta, q.zeta, hbuf[8 * i + 2]);
                q.lu_first = false;
                if (q.zeta >= 1.0) {
                    q.l += 1;
                    std::swap(q.Glo, q.Ghi);
                    std::swap(q.plo, q.phi);
                    q.in_lu = false;
                    q.prev_lu = true;
                }
            } else {
                r.solves[q.l] += q.J * cfg->n_mcmc;
                q.beta = q.t_next;
                log_stage(r, q.checked ? 1 : 0, q.l, q.beta, 0.0, hbuf[8 * i + 2]);
                q.prev_lu = false;
            }
            ++q.stage;
        }
    }
    for (int i = 0; i < n_inst; ++i) {
        Inst& q = I[i];
        res[i].final_level = q.l;
        res[i].final_beta = q.beta;
        MLS_CHECK_HIP(hipMemcpyAsync(q.out, q.theta, sizeof(double) * q.J * K, hipMemcpyDeviceToDevice, s));
        MLS_CHECK_HIP(hipMemcpyAsync(hbuf + 8 * i + 4, q.counters, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    }
    MLS_CHECK_HIP(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < n_inst; ++i) {
        int64_t a;
        std::memcpy(&a, hbuf + 8 * i + 4, sizeof(a));
        res[i].accepted = a;
        res[i].seconds = secs;
        res[i].graphs_launched = graphs;
    }
    return rc;
}
