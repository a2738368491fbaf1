// Internal declarations of the MI355X MLS^2MC library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mls2mc.h"

namespace mls {

constexpr int kMaxLevel = 10;

// ---------------------------------------------------------------- errors --
void set_error(const std::string& msg);

struct Status {
    int code = MLS2MC_OK;
};

#define MLS_CHECK_HIP(expr)                                                          \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::mls::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));     \
            return MLS2MC_EDEVICE;                                                   \
        }                                                                            \
    } while (0)

#define MLS_REQUIRE(cond, msg)                                                       \
    do {                                                                             \
        if (!(cond)) {                                                               \
            ::mls::set_error(msg);                                                   \
            return MLS2MC_EINVAL;                                                    \
        }                                                                            \
    } while (0)

#define MLS_TRY(expr)                                                                \
    do {                                                                             \
        int rc_ = (expr);                                                            \
        if (rc_ != MLS2MC_OK) return rc_;                                            \
    } while (0)

// ------------------------------------------------------- device buffers --
// Grow-only device allocation owned by the context.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t want);
    void release();
    template <typename T>
    T* as() const { return static_cast<T*>(ptr); }
};

// ------------------------------------------------------------- sizes --
inline int64_t n_side(int l) { return int64_t(1) << l; }
inline int64_t n_elem(int l) { return 2 * n_side(l) * n_side(l); }
inline int64_t n_unk(int l) { return (n_side(l) - 1) * (n_side(l) - 1); }
inline int64_t n_pad(int l) { return (n_side(l) + 1) * (n_side(l) + 1); }

// Per-particle solver workspace (elements of the working type), see solver.hip.
int64_t solver_slot_elems(int l, bool mixed);
// LDS elements the solver's residency policy uses at level l for a budget
int64_t solver_lds_elems_used(int l, bool mixed, int64_t budget_elems);

// ------------------------------------------------------- observation --
// Three nodes (padded-grid offsets) and barycentric weights per observation.
struct ObsTable {
    int32_t* idx = nullptr;  // device, 3 * nobs
    double* w = nullptr;     // device, 3 * nobs
};

// ---------------------------------------------------------- profiling --
struct ProfRec {
    hipEvent_t a = nullptr, b = nullptr;
};
struct ProfSlot {
    std::vector<ProfRec> recs;
    int64_t items = 0;
};

struct Surrogate;
void surrogate_destroy(mls2mc_ctx* ctx);

// --------------------------------------------------------------- ctx --
}  // namespace mls

struct mls2mc_ctx {
    mls2mc_problem prob;
    int device = 0;
    int nobs = 0;
    // KL modes (host): sqrt(lambda_k), per-direction frequency, amplitude
    // ratio omega/c and inverse L2 norm of the 1-D factor
    std::vector<double> sqrt_lam, om_x, om_y, amp_x, amp_y, inv_x, inv_y;
    double* d_modes = nullptr;                        // 7*K doubles on device
    double* d_B[mls::kMaxLevel + 1] = {};             // K x n_e FP64 bases
    __hip_bfloat16* d_B16[mls::kMaxLevel + 1] = {};   // K x n_e BF16 bases (mixed)
    mls::ObsTable obs[mls::kMaxLevel + 1];
    // scratch
    mls::DevBuf ws_solver;   // solver slots
    mls::DevBuf ws_kappa;    // KL field output for forward()
    mls::DevBuf ws_theta16;  // BF16 copy of theta (mixed)
    mls::DevBuf ws_misc;     // sampler scratch
    mls::DevBuf ws_pcn;      // pCN proposals and their G / phi
    mls::DevBuf ws_status;   // int8 status + int32 iters for internal forwards
    mls::DevBuf ws_run;      // state of mls2mc_run
    int n_cu = 256;                             // compute units of the device
    int solver_grid[mls::kMaxLevel + 1] = {};  // persistent grid per level (0 = auto)
    int solver_block[mls::kMaxLevel + 1] = {};
    int solver_nu[mls::kMaxLevel + 1] = {};     // Gauss-Seidel sweeps per V-cycle side (0 = 1)
    int solver_lds[mls::kMaxLevel + 1] = {};    // LDS budget in bytes (0 = 64 KiB, -1 = none)
    int max_lds = 65536;                        // largest LDS budget a launch may take (bytes)
    int list_grid = 0, list_block = 0;          // work-list launch shape (0 = auto)
    double rtol = 1e-11;
    int max_iters = 200;
    // instrumentation (see mls2mc_profile)
    bool prof_on = false;
    mls::ProfSlot prof[2][mls::kMaxLevel + 1];
    int64_t* d_prof_iters = nullptr;  // [kMaxLevel+1][2] device counters
    mls::DevBuf ws_prof;              // iteration scratch when the caller passes none
    mls::Surrogate* sur = nullptr;    // learned surrogate (mlp.hip)
    mls::DevBuf ws_da;                // delayed-acceptance scratch
    mls::DevBuf ws_list;              // device copies of work lists
    mls::DevBuf ws_batch;             // state of mls2mc_run_batch
    void* h_list = nullptr;           // pinned host staging of work lists
    size_t h_list_bytes = 0;
    hipEvent_t h_list_ev = nullptr;   // last copy out of h_list
    int64_t* d_chunk_count = nullptr; // per-chunk device counts
    unsigned long long* d_queue = nullptr;  // the solver's particle counter and finished-workgroup count
    double* d_lin_A = nullptr;        // linear test model (N_obs x K each), or null
    double* d_lin_E = nullptr;
    double* d_sur_S = nullptr;        // linear surrogate G~ = S theta (N_obs x K), or null: the network
    double* da_err = nullptr;         // while mls2mc_run runs with the surrogate: accumulator of the
                                      // surrogate's error against stage-2 solves {sum, max, count}
};

namespace mls {

// ------------------------------------------------------------ launchers --
int build_kl_tables(mls2mc_ctx* ctx);
int build_matern_tables(mls2mc_ctx* ctx);  // kl_matern.hip
int launch_kl_field(mls2mc_ctx* ctx, int l, int64_t N, const double* theta, void* out, int kind,
                    hipStream_t s, const int64_t* N_dev = nullptr);
int build_obs_tables(mls2mc_ctx* ctx);

struct SolveArgs {
    int l = 0;
    int64_t N = 0;
    const void* kappa = nullptr;  // N x n_e (double, or float for mixed)
    bool kappa_f32 = false;
    double* G = nullptr;          // N x nobs
    double* p_out = nullptr;      // N x M or null
    int8_t* status = nullptr;     // N or null
    int32_t* iters = nullptr;     // N or null
    const double* y = nullptr;    // fused potential (null: off)
    double* phi = nullptr;
    const int64_t* N_dev = nullptr;  // device-side count <= N (null: N)
};
int launch_solve(mls2mc_ctx* ctx, const SolveArgs& a, hipStream_t s);
// flow-cell problem (flowcell.hip): its solver and its unknowns per level
int launch_flow_solve(mls2mc_ctx* ctx, const SolveArgs& a, hipStream_t s);
int64_t flow_unknowns(int l);

// one entry of a fused multi-instance / multi-level solver launch
struct SolveItem {
    int l;
    int64_t N;
    int64_t base;        // sum of N over the items before this one
    const void* kappa;   // N x n_e(l)
    double* G;           // N x nobs
    double* phi;         // N or null (fused potential with y)
    const double* y;
    int8_t* status;      // N or null
    int32_t* iters;      // N or null
};
int launch_solve_list(mls2mc_ctx* ctx, const SolveItem* items_dev, int n_items, int64_t total, int lmax,
                      bool mixed, hipStream_t s);

// one entry of a grouped KL GEMM launch (64 x 64 output tiles)
struct GemmItem {
    const double* theta;          // N x K
    const double* B;              // K x n_e (FP64 basis of the level)
    const __hip_bfloat16* B16;    // n_e x Kp (BF16 basis, mixed)
    void* out;                    // N x n_e kappa (double, or float for mixed)
    int64_t N, ne;
    int64_t tile_base;            // tiles of the items before this one
    int64_t tiles_x;              // ceil(ne / 64)
};
int launch_kl_list(mls2mc_ctx* ctx, const GemmItem* items_dev, int n_items, int64_t total_tiles, hipStream_t s);
// build and enqueue one fused forward over many (level, theta) items
struct FwdItem {
    int l;
    int64_t N;
    const double* theta;
    double* G;
    const double* y;
    double* phi;
    int8_t* status;
    int32_t* iters;
};
int forward_list(mls2mc_ctx* ctx, const std::vector<FwdItem>& items, hipStream_t s);
struct ListChunk {  // one prepared (grouped GEMM, work-list solve) pair
    const GemmItem* gemm;
    const SolveItem* solve;
    int n;
    int64_t tiles, total;
    int lmax;
};
int prepare_list(mls2mc_ctx* ctx, const std::vector<FwdItem>& items, std::vector<ListChunk>& out, hipStream_t s);
int enqueue_list(mls2mc_ctx* ctx, const std::vector<ListChunk>& chunks, hipStream_t s);

int launch_loglik(mls2mc_ctx* ctx, int64_t N, const double* G, const double* y, double* phi,
                  hipStream_t s);
int launch_next_step(mls2mc_ctx* ctx, int64_t N, const double* d, double scale, double cur,
                     double tau, double eps, double* out3, double* logw, double* w, hipStream_t s);
int launch_resample(mls2mc_ctx* ctx, int64_t N, const double* w, const double* u, int32_t* anc,
                    hipStream_t s);
int launch_resample_into(int64_t N, const double* w, const double* u, uint64_t* C, int32_t* anc,
                         hipStream_t s);
int launch_gather(int64_t N, int64_t ncols, const int32_t* anc, int64_t n_src, const double* src,
                  double* dst, hipStream_t s);
int launch_philox(uint64_t seed, uint32_t stream_id, uint32_t stage, uint32_t sub, int64_t n,
                  int normal, double* out, hipStream_t s);
int launch_pcn_propose(int64_t N, int K, double s_pcn, int kernel, const double* theta, const double* xi,
                       double* out, hipStream_t s);
int launch_pcn_accept(int64_t N, int K, int nobs, int mode, int rwm, double beta, double zeta,
                      const double* u, const double* th_new, const double* Glo_new,
                      const double* Ghi_new, const double* plo_new, const double* phi_new,
                      const int8_t* st_lo, const int8_t* st_hi, double* theta, double* Glo,
                      double* Ghi, double* plo, double* phi, uint8_t* acc, hipStream_t s);
int launch_ess_cv(int64_t N, const double* dlo, const double* dhi, double scale, double* out,
                  hipStream_t s);
int launch_reduce_i32(int64_t N, const int32_t* v, const int8_t* st, int64_t* out2,
                      hipStream_t s);
int launch_linear_map(int64_t N, int K, int nobs, const double* S, const double* theta, double* G,
                      hipStream_t s);
int launch_linear_forward(mls2mc_ctx* ctx, int l, int64_t N, const double* theta, double* G,
                          int8_t* status, int32_t* iters, const double* y, double* phi,
                          hipStream_t s, const int64_t* N_dev);
int launch_d2f(const double* a, float* b, int64_t n, hipStream_t s);
int prof_begin(mls2mc_ctx* ctx, int kclass, int l, int64_t items, hipStream_t s, ProfRec* rec);
int prof_end(mls2mc_ctx* ctx, int kclass, int l, const ProfRec& rec, hipStream_t s);

int forward_theta(mls2mc_ctx* ctx, int l, int64_t N, const double* theta, double* G,
                  int8_t* status, int32_t* iters, const double* y, double* phi, hipStream_t s,
                  const int64_t* N_dev = nullptr);

// --------------------------------------------------- device utilities --
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// A value every lane of the wave holds bitwise alike, moved to scalar
// registers (frees vector registers in the large solver kernels).
__device__ __forceinline__ double wave_uniform(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Deterministic block reduction (fixed butterfly within waves, waves summed
// in order by every thread).  `red` must hold BS/64 doubles; the result is
// returned to all threads.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double* red)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < BS / 64; ++k) s += red[k];
    __syncthreads();
    return wave_uniform(s);  // every thread summed the same terms in the same order
}

template <int BS>
__device__ __forceinline__ double block_max(double v, double* red)
{
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int k = 1; k < BS / 64; ++k) s = fmax(s, red[k]);
    __syncthreads();
    return wave_uniform(s);
}

}  // namespace mls
