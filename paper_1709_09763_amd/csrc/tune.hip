// Launch-shape autotuner for the persistent solver: for one level and batch
// size it times candidate (workgroups, block size) pairs on prior draws and
// keeps the fastest.  The choice trades slot-workspace residency in the
// caches (fewer slots) against latency hiding (more workgroups per CU).
#include <algorithm>
#include <vector>

#include "common.h"

namespace mls {

static int time_solve(mls2mc_ctx* ctx, const SolveArgs& a, hipStream_t s, int reps, float* best_ms)
{
    hipEvent_t e0, e1;
    MLS_CHECK_HIP(hipEventCreate(&e0));
    MLS_CHECK_HIP(hipEventCreate(&e1));
    MLS_TRY(launch_solve(ctx, a, s));  // warm: workspace and caches
    float best = 1e30f;
    for (int r = 0; r < reps; ++r) {
        MLS_CHECK_HIP(hipEventRecord(e0, s));
        MLS_TRY(launch_solve(ctx, a, s));
        MLS_CHECK_HIP(hipEventRecord(e1, s));
        MLS_CHECK_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        MLS_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *best_ms = best;
    return MLS2MC_OK;
}

}  // namespace mls

using namespace mls;

extern "C" int mls2mc_set_launch(mls2mc_ctx* ctx, int l, int grid, int block, int nu, int lds_bytes)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(l >= 1 && l <= kMaxLevel, "set_launch: bad level");
    MLS_REQUIRE(grid >= 0 && grid <= (1 << 20), "set_launch: grid outside [0, 2^20]");
    MLS_REQUIRE(block == 0 || block == 64 || block == 128 || block == 256 || block == 512 ||
                    block == 1024,
                "set_launch: block must be 0 (auto), 64, 128, 256, 512 or 1024");
    MLS_REQUIRE(nu >= 0 && nu <= 4, "set_launch: nu must be 0 (default 1) .. 4");
    MLS_REQUIRE(lds_bytes == -1 || (lds_bytes >= 0 && lds_bytes <= ctx->max_lds),
                "set_launch: lds_bytes must be -1 (none), 0 (default 64 KiB) or up to the device's "
                "LDS per workgroup less 1 KiB");
    ctx->solver_grid[l] = grid;
    ctx->solver_block[l] = block;
    ctx->solver_nu[l] = nu;
    ctx->solver_lds[l] = lds_bytes;
    return MLS2MC_OK;
}

extern "C" int mls2mc_get_launch(const mls2mc_ctx* ctx, int l, int* grid, int* block, int* nu, int* lds_bytes)
{
    MLS_REQUIRE(ctx && grid && block && nu && lds_bytes, "get_launch: null argument");
    MLS_REQUIRE(l >= 1 && l <= kMaxLevel, "get_launch: bad level");
    *grid = ctx->solver_grid[l];
    *block = ctx->solver_block[l];
    *nu = ctx->solver_nu[l];
    *lds_bytes = ctx->solver_lds[l];
    return MLS2MC_OK;
}

extern "C" int mls2mc_autotune(mls2mc_ctx* ctx, int l, int64_t N, double* best_ms, void* stream)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(l >= ctx->prob.l_min && l <= ctx->prob.l_max, "autotune: level outside the context");
    MLS_REQUIRE(N >= 1 && N <= (int64_t(1) << 20), "autotune: need 1 <= N <= 2^20");
    const hipStream_t s = (hipStream_t)stream;
    const bool mixed = ctx->prob.precision == MLS2MC_MIXED;
    const int K = ctx->prob.K, nobs = ctx->nobs;
    const int64_t ne = n_elem(l);
    const size_t esz = mixed ? sizeof(float) : sizeof(double);
    // private buffers: theta, kappa, G
    DevBuf th, kap, G;
    int rc = th.ensure(sizeof(double) * (size_t)N * K);
    if (rc == MLS2MC_OK) rc = kap.ensure(esz * (size_t)N * ne);
    if (rc == MLS2MC_OK) rc = G.ensure(sizeof(double) * (size_t)N * nobs);
    if (rc == MLS2MC_OK) rc = launch_philox(0x5eedull, 0, 0, 0, N * K, 1, th.as<double>(), s);
    if (rc == MLS2MC_OK)
        rc = launch_kl_field(ctx, l, N, th.as<double>(), kap.ptr,
                             mixed ? MLS2MC_FIELD_KAPPA_F32 : MLS2MC_FIELD_KAPPA_F64, s);
    const bool prof = ctx->prof_on;
    ctx->prof_on = false;
    SolveArgs a;
    a.l = l;
    a.N = N;
    a.kappa = kap.ptr;
    a.kappa_f32 = mixed;
    a.G = G.as<double>();
    const int cu = ctx->n_cu;
    std::vector<int> wpc, blocks;
    if (l <= 4) { wpc = {1, 2, 4, 8, 16}; blocks = {64, 128, 256}; }
    else if (l <= 6) { wpc = {1, 2, 4, 8}; blocks = {128, 256, 512}; }
    else { wpc = {1, 2, 4}; blocks = {256, 512, 1024}; }
    // LDS budgets: none, the default 64 KiB, 80 KiB (still two workgroups per
    // CU on a 160 KiB LDS) and the device maximum; a budget that gives the
    // same residency as a smaller one is skipped
    std::vector<int> ldsc = {-1, 0};
    {
        const int64_t esz_ = (int64_t)esz;
        int64_t last = solver_lds_elems_used(l, mixed, 65536 / esz_);
        for (int b : {81920, ctx->max_lds}) {
            if (b > ctx->max_lds || b <= 65536) continue;
            const int64_t u = solver_lds_elems_used(l, mixed, b / esz_);
            if (u > last) { ldsc.push_back(b); last = u; }
        }
    }
    float best = 1e30f;
    int bg = 0, bb = 0, bn = 1, bl = 0;
    for (int lds : ldsc) {
        ctx->solver_lds[l] = lds;
        for (int nu = 1; nu <= 2; ++nu) {
            ctx->solver_nu[l] = nu;
            for (int b : blocks) {
                if (rc != MLS2MC_OK) break;
                int64_t last_grid = -1;
                for (int w : wpc) {
                    int64_t g = std::min<int64_t>((int64_t)w * cu, N);
                    if (g == last_grid) continue;
                    last_grid = g;
                    ctx->solver_grid[l] = (int)g;
                    ctx->solver_block[l] = b;
                    float ms = 0.f;
                    rc = time_solve(ctx, a, s, 3, &ms);
                    if (rc != MLS2MC_OK) break;
                    if (ms < best) { best = ms; bg = (int)g; bb = b; bn = nu; bl = lds; }
                }
            }
        }
    }
    ctx->prof_on = prof;
    ctx->solver_grid[l] = bg;
    ctx->solver_block[l] = bb;
    ctx->solver_nu[l] = bn;
    ctx->solver_lds[l] = bl;
    th.release();
    kap.release();
    G.release();
    if (best_ms) *best_ms = best;
    return rc;
}
