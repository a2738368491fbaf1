// Matern (smoothness 3/2) prior covariance and its truncated Karhunen-Loeve
// expansion by the Nystrom method: the prior of the paper's elliptic
// examples (Sec. 5), a Matern field truncated to its leading KL terms.
//
//   C(r) = sigma2 (1 + sqrt(6) r / lam) exp(-sqrt(6) r / lam)
//
// (Bessel argument 2 sqrt(nu) r / lam; the variance fractions the paper prints
// for its examples hold under this form).  The operator is discretised by the
// midpoint rule on an m x m grid of the unit square, points P_q = ((a+1/2)/m,
// (b+1/2)/m), q = b m + a, weights w = 1/m^2, giving A = w [C(|P_q - P_q'|)].
//
// A commutes with the reflections x1 -> 1 - x1 and x2 -> 1 - x2, so it splits
// into four parity classes (+,+), (-,+), (+,-), (-,-) of (m/2)^2 unknowns each;
// (+,-) is (-,+) with the coordinates swapped.  The three distinct classes are
// solved separately, one host thread each, by subspace iteration with
// Rayleigh-Ritz: the block products A V run on the GPU, the
// orthonormalisation and the small dense eigenproblems on the host.  The eigenvectors are then canonical: parity
// definite, swapped pairs with identical eigenvalues in class order, sign
// fixed by a quadratic Weyl sequence (a linear one is nearly constant over
// the square's reflection orbits and cannot fix the sign of every mode).  The basis at the element centroids is the
// Nystrom extension
//   B_l[k, e] = sqrt(lambda_k) phi_k(c_e) = sqrt(w / lambda_k) sum_q C(|c_e - P_q|) v_k[q],
// a K x M by M x n_e contraction with the kernel matrix generated on the fly,
// on the FP64 matrix cores.
#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "common.h"

namespace mls {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr double kGoldenFrac = 0.6180339887498949;  // sign rule weights g_q = frac((q+1)^2 * this) - 1/2
constexpr double kResTol = 1e-13;                  // Ritz residual / largest eigenvalue at convergence
constexpr double kResAccept = 1e-11;               // accepted when the residual no longer falls
constexpr int kPowerSteps = 6;                     // subspace steps between Rayleigh-Ritz steps
constexpr int kMaxSteps = 600;

struct TmpBuf {
    DevBuf b;
    ~TmpBuf() { b.release(); }
};

__device__ __forceinline__ double matern32(double r, double sc, double sigma2)
{
    const double a = sc * r;
    return sigma2 * (1.0 + a) * exp(-a);
}

// A_s[p, p'] = w sum_h chi(h) C(|P_p - P_{h p'}|), h in {I, Fx, Fy, FxFy}; p = b h + a
// over the representatives a, b < m/2.  Row p = blockIdx.y.
__global__ void matern_class_kernel(int m, double sc, double s2w, int sx, int sy, double* __restrict__ A)
{
    const int h = m / 2, nb = h * h;
    const int q = blockIdx.x * blockDim.x + threadIdx.x, p = blockIdx.y;
    if (q >= nb) return;
    const double x = (p % h + 0.5) / m, y = (p / h + 0.5) / m;
    const double xq = (q % h + 0.5) / m, yq = (q / h + 0.5) / m;
    const double dx0 = x - xq, dx1 = x - (1.0 - xq), dy0 = y - yq, dy1 = y - (1.0 - yq);
    double v = matern32(sqrt(dx0 * dx0 + dy0 * dy0), sc, 1.0);
    v += sx * matern32(sqrt(dx1 * dx1 + dy0 * dy0), sc, 1.0);
    v += sy * matern32(sqrt(dx0 * dx0 + dy1 * dy1), sc, 1.0);
    v += sx * sy * matern32(sqrt(dx1 * dx1 + dy1 * dy1), sc, 1.0);
    A[(int64_t)p * nb + q] = s2w * v;
}

// W = A V for a symmetric nb x nb A (row-major) and column-major nb x s
// blocks V, W.  16 x 16 output tiles through LDS.
__global__ __launch_bounds__(256) void sym_block_product(int nb, int s, const double* __restrict__ A,
                                                         const double* __restrict__ V, double* __restrict__ W)
{
    __shared__ double As[16][17], Vs[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = blockIdx.y * 16 + ty;  // row of W
    const int j = blockIdx.x * 16 + tx;  // column of W
    const int jl = blockIdx.x * 16 + ty; // column loaded by this thread
    double acc = 0.0;
    for (int k0 = 0; k0 < nb; k0 += 16) {
        As[ty][tx] = (i < nb && k0 + tx < nb) ? A[(int64_t)i * nb + k0 + tx] : 0.0;
        Vs[ty][tx] = (jl < s && k0 + tx < nb) ? V[(int64_t)jl * nb + k0 + tx] : 0.0;  // Vs[col][k]
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) acc += As[ty][kk] * Vs[tx][kk];
        __syncthreads();
    }
    if (i < nb && j < s) W[(int64_t)j * nb + i] = acc;
}

// B[k, e] = sum_q Vs[k, q] C(|c_e - P_q|) on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64), the kernel operand generated per lane.  A
// workgroup of four waves computes 64 modes x 64 elements; wave w owns modes
// 16w..16w+15.  Lane layout as in the KL GEMM: A[i][k] with i = lane%16,
// k = lane/16; B[k][j] with j = lane%16; lane holds D[lane/16 + 4v][lane%16].
__global__ __launch_bounds__(256) void nystrom_extend_kernel(const double* __restrict__ Vs, int K, int m,
                                                             double sc, double sigma2, int l,
                                                             double* __restrict__ B)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int64_t ne = int64_t(2) << (2 * l);
    const int n = 1 << l;
    const int64_t e0 = (int64_t)blockIdx.x * 64;
    const int k0 = blockIdx.y * 64 + wv * 16;
    const int M = m * m;
    double cx[4], cy[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {  // centroids of this lane's four elements
        const int64_t e = min(e0 + c * 16 + r, ne - 1);
        const int64_t cell = e >> 1;
        const int i = (int)(cell & (n - 1)), j = (int)(cell >> l);
        if ((e & 1) == 0) {
            cx[c] = (double)(3 * i + 2) / (double)(3 * n);
            cy[c] = (double)(3 * j + 1) / (double)(3 * n);
        } else {
            cx[c] = (double)(3 * i + 1) / (double)(3 * n);
            cy[c] = (double)(3 * j + 2) / (double)(3 * n);
        }
    }
    dbl4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int krow = k0 + r;
    const double* vrow = Vs + (int64_t)min(krow, K - 1) * M;
    for (int q0 = 0; q0 < M; q0 += 4) {
        const int q = q0 + kq;
        const double a = krow < K ? vrow[q] : 0.0;
        const double px = (q % m + 0.5) / m, py = (q / m + 0.5) / m;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double dx = cx[c] - px, dy = cy[c] - py;
            const double b = matern32(sqrt(dx * dx + dy * dy), sc, sigma2);
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int k = k0 + kq + 4 * v;
            const int64_t e = e0 + c * 16 + r;
            if (k < K && e < ne) B[(int64_t)k * ne + e] = acc[c][v];
        }
}

// BF16 copy of a K x n_e basis, transposed to n_e x Kp (K padded with zeros)
__global__ void basis_to_bf16(const double* __restrict__ B, int K, int Kp, int64_t ne,
                              __hip_bfloat16* __restrict__ Bt)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= ne) return;
    for (int k = 0; k < Kp; ++k)
        Bt[e * Kp + k] = __float2bfloat16(k < K ? (float)B[(int64_t)k * ne + e] : 0.f);
}

// ------------------------------------------------------------ host dense --
struct Rng {  // splitmix64
    uint64_t s;
    double uniform()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    }
};

double dot(const double* a, const double* b, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

// Orthonormalise the columns of the column-major n x s block in place:
// Gram-Schmidt, each column projected twice; a column that (nearly) lies in
// the span of the previous ones is replaced by a random one.
void orthonormalise(std::vector<double>& W, int n, int s, Rng& rng)
{
    for (int j = 0; j < s; ++j) {
        double* w = &W[(size_t)j * n];
        for (int attempt = 0; attempt < 4; ++attempt) {
            const double n0 = std::sqrt(dot(w, w, n));
            for (int pass = 0; pass < 2; ++pass)
                for (int i = 0; i < j; ++i) {
                    const double* q = &W[(size_t)i * n];
                    const double c = dot(q, w, n);
                    for (int t = 0; t < n; ++t) w[t] -= c * q[t];
                }
            const double nn = std::sqrt(dot(w, w, n));
            if (nn > 1e-10 * n0 && nn > 0.0) {
                for (int t = 0; t < n; ++t) w[t] /= nn;
                break;
            }
            for (int t = 0; t < n; ++t) w[t] = rng.uniform();
        }
    }
}

// Eigen-decomposition of the symmetric s x s H (column-major) by cyclic
// Jacobi rotations: theta descending, U column-major with U[:, k] the
// eigenvector of theta[k].
void jacobi_eigen(std::vector<double> H, int s, std::vector<double>& theta, std::vector<double>& U)
{
    std::vector<double> Z((size_t)s * s, 0.0);
    for (int i = 0; i < s; ++i) Z[(size_t)i * s + i] = 1.0;
    auto h = [&](int i, int j) -> double& { return H[(size_t)j * s + i]; };
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int j = 0; j < s; ++j) {
            diag += h(j, j) * h(j, j);
            for (int i = 0; i < j; ++i) off += h(i, j) * h(i, j);
        }
        if (off <= 1e-34 * diag) break;
        for (int p = 0; p < s - 1; ++p)
            for (int q = p + 1; q < s; ++q) {
                const double apq = h(p, q);
                if (apq == 0.0) continue;
                const double app = h(p, p), aqq = h(q, q);
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
                for (int k = 0; k < s; ++k) {  // columns p, q
                    const double hkp = h(k, p), hkq = h(k, q);
                    h(k, p) = c * hkp - sn * hkq;
                    h(k, q) = sn * hkp + c * hkq;
                }
                for (int k = 0; k < s; ++k) {  // rows p, q
                    const double hpk = h(p, k), hqk = h(q, k);
                    h(p, k) = c * hpk - sn * hqk;
                    h(q, k) = sn * hpk + c * hqk;
                }
                h(p, q) = h(q, p) = 0.0;
                double* zp = &Z[(size_t)p * s];
                double* zq = &Z[(size_t)q * s];
                for (int k = 0; k < s; ++k) {
                    const double a = zp[k], b = zq[k];
                    zp[k] = c * a - sn * b;
                    zq[k] = sn * a + c * b;
                }
            }
    }
    std::vector<int> ord(s);
    for (int i = 0; i < s; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return h(a, a) > h(b, b); });
    theta.resize(s);
    U.assign((size_t)s * s, 0.0);
    for (int k = 0; k < s; ++k) {
        theta[k] = h(ord[k], ord[k]);
        std::copy(&Z[(size_t)ord[k] * s], &Z[(size_t)ord[k] * s] + s, &U[(size_t)k * s]);
    }
}

// C = A U for column-major n x s A and s x t U
void times_small(const std::vector<double>& A, int n, int s, const std::vector<double>& U, int t,
                 std::vector<double>& C)
{
    C.assign((size_t)n * t, 0.0);
    for (int j = 0; j < t; ++j) {
        double* c = &C[(size_t)j * n];
        for (int k = 0; k < s; ++k) {
            const double u = U[(size_t)j * s + k];
            if (u == 0.0) continue;
            const double* a = &A[(size_t)k * n];
            for (int i = 0; i < n; ++i) c[i] += u * a[i];
        }
    }
}

struct ClassSol {
    int n = 0;                // eigenpairs kept (converged)
    std::vector<double> lam;  // n, descending
    std::vector<double> vec;  // nb x n column-major, orthonormal
};

// The `need` leading eigenpairs of the parity class (sx, sy).
int solve_class(int m, double sc, double s2w, int sx, int sy, int need, uint64_t seed, ClassSol& out)
{
    const int h = m / 2, nb = h * h;
    need = std::min(need, nb);
    const int s = std::min(nb, need + std::max(10, need / 2));
    TmpBuf dA, dV, dW;
    MLS_TRY(dA.b.ensure(sizeof(double) * (size_t)nb * nb));
    MLS_TRY(dV.b.ensure(sizeof(double) * (size_t)nb * s));
    MLS_TRY(dW.b.ensure(sizeof(double) * (size_t)nb * s));
    double* A = dA.b.as<double>();
    {
        dim3 g((unsigned)((nb + 255) / 256), (unsigned)nb);
        matern_class_kernel<<<g, 256>>>(m, sc, s2w, sx, sy, A);
        MLS_CHECK_HIP(hipGetLastError());
    }
    Rng rng{seed};
    std::vector<double> V((size_t)nb * s), W, theta, U, X, AX;
    for (auto& v : V) v = rng.uniform();
    orthonormalise(V, nb, s, rng);
    const dim3 pg((unsigned)((s + 15) / 16), (unsigned)((nb + 15) / 16));
    auto apply = [&](std::vector<double>& in, std::vector<double>& res) -> int {
        MLS_CHECK_HIP(hipMemcpy(dV.b.ptr, in.data(), sizeof(double) * in.size(), hipMemcpyHostToDevice));
        sym_block_product<<<pg, 256>>>(nb, s, A, dV.b.as<double>(), dW.b.as<double>());
        MLS_CHECK_HIP(hipGetLastError());
        res.resize((size_t)nb * s);
        MLS_CHECK_HIP(hipMemcpy(res.data(), dW.b.ptr, sizeof(double) * res.size(), hipMemcpyDeviceToHost));
        return MLS2MC_OK;
    };
    double prev = HUGE_VAL;
    for (int step = 0;; ++step) {
        MLS_TRY(apply(V, W));  // W = A V, V orthonormal
        if (step % kPowerSteps == kPowerSteps - 1 || s == nb || step + 1 >= kMaxSteps) {
            // Rayleigh-Ritz on span(V): H = V^T A V
            std::vector<double> H((size_t)s * s);
            for (int j = 0; j < s; ++j)
                for (int i = 0; i <= j; ++i)
                    H[(size_t)j * s + i] = H[(size_t)i * s + j] =
                        0.5 * (dot(&V[(size_t)i * nb], &W[(size_t)j * nb], nb) +
                               dot(&V[(size_t)j * nb], &W[(size_t)i * nb], nb));
            jacobi_eigen(H, s, theta, U);
            times_small(V, nb, s, U, s, X);   // Ritz vectors
            times_small(W, nb, s, U, s, AX);  // A times them
            double res = 0.0;
            for (int k = 0; k < need; ++k) {
                double r2 = 0.0;
                const double* x = &X[(size_t)k * nb];
                const double* ax = &AX[(size_t)k * nb];
                for (int i = 0; i < nb; ++i) {
                    const double d = ax[i] - theta[k] * x[i];
                    r2 += d * d;
                }
                res = std::max(res, std::sqrt(r2));
            }
            res /= std::fabs(theta[0]);
            const bool done = res <= kResTol || s == nb || (res <= kResAccept && res > 0.7 * prev);
            if (done) {
                out.n = need;
                out.lam.assign(theta.begin(), theta.begin() + need);
                out.vec.assign(X.begin(), X.begin() + (size_t)need * nb);
                return MLS2MC_OK;
            }
            if (step + 1 >= kMaxSteps) {
                set_error("create: Matern KL eigensolver did not converge");
                return MLS2MC_ENOTCONV;
            }
            prev = res;
            V.swap(X);
            orthonormalise(V, nb, s, rng);  // Ritz vectors are orthonormal up to rounding
        } else {
            V.swap(W);
            orthonormalise(V, nb, s, rng);
        }
    }
}

}  // namespace

int build_matern_tables(mls2mc_ctx* ctx)
{
    const mls2mc_problem& p = ctx->prob;
    const int m = p.kl_quad ? p.kl_quad : 64;
    MLS_REQUIRE(m >= 4 && m <= 128 && m % 2 == 0, "create: kl_quad must be even, 4..128");
    const int M = m * m, h = m / 2, nb = h * h, K = p.K;
    MLS_REQUIRE(K <= M, "create: K exceeds the Nystrom grid's m*m eigenpairs");
    const double sc = std::sqrt(6.0) / p.corr_len, w = 1.0 / ((double)m * m);
    const int cls_sx[4] = {1, -1, 1, -1}, cls_sy[4] = {1, 1, -1, -1};
    // classes 0, 1, 3 are solved; 2 is class 1 with the coordinates swapped
    ClassSol sol[4];
    int need[4] = {0, 0, 0, 0};
    for (int c : {0, 1, 3}) need[c] = std::min(nb, (K * 5 + 15) / 16 + 8);
    bool todo[4] = {true, true, false, true};
    struct Cand { double lam; int cls, j; };
    std::vector<Cand> cand;
    for (int round = 0; round < 16; ++round) {
        // the classes are independent: one host thread each (the current
        // device and the error message are per thread)
        int rcs[4] = {MLS2MC_OK, MLS2MC_OK, MLS2MC_OK, MLS2MC_OK};
        std::string errs[4];
        std::vector<std::thread> workers;
        for (int c : {0, 1, 3})
            if (todo[c])
                workers.emplace_back([&, c]() {
                    if (hipSetDevice(ctx->device) != hipSuccess) {
                        rcs[c] = MLS2MC_EDEVICE;
                        errs[c] = "create: hipSetDevice failed in a Matern KL worker";
                        return;
                    }
                    rcs[c] = solve_class(m, sc, p.sigma2 * w, cls_sx[c], cls_sy[c], need[c],
                                         0x6d61746572ull + 977u * (unsigned)c + 131u * (unsigned)need[c], sol[c]);
                    if (rcs[c] != MLS2MC_OK) errs[c] = mls2mc_last_error();
                });
        for (auto& t : workers) t.join();
        for (int c : {0, 1, 3}) {
            if (rcs[c] != MLS2MC_OK) {
                set_error(errs[c]);
                return rcs[c];
            }
            todo[c] = false;
        }
        cand.clear();
        for (int c : {0, 1, 3})
            for (int j = 0; j < sol[c].n; ++j) {
                cand.push_back({sol[c].lam[j], c, j});
                if (c == 1) cand.push_back({sol[c].lam[j], 2, j});
            }
        std::sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
            if (a.lam != b.lam) return a.lam > b.lam;
            return a.cls < b.cls;
        });
        bool complete = (int)cand.size() >= K;
        const double t = complete ? cand[K - 1].lam : 0.0;
        for (int c : {0, 1, 3}) {
            const bool short_c = (int)cand.size() < K || sol[c].lam[sol[c].n - 1] > t;
            if (short_c && sol[c].n < nb) {
                need[c] = std::min(nb, 2 * need[c]);
                todo[c] = true;
                complete = false;
            }
        }
        if (complete) break;
        MLS_REQUIRE(round < 15, "create: Matern KL could not isolate the leading eigenpairs");
    }
    // canonical full-grid eigenvectors, scaled for the Nystrom extension
    std::vector<double> Vs((size_t)K * M);
    ctx->sqrt_lam.resize(K);
    for (int k = 0; k < K; ++k) {
        const Cand& cd = cand[k];
        const int src = cd.cls == 2 ? 1 : cd.cls;
        const double* v = &sol[src].vec[(size_t)cd.j * nb];
        const int sx = cls_sx[cd.cls], sy = cls_sy[cd.cls];
        double* out = &Vs[(size_t)k * M];
        for (int b = 0; b < m; ++b)
            for (int a = 0; a < m; ++a) {
                const int ar = a < h ? a : m - 1 - a, br = b < h ? b : m - 1 - b;
                const double sg = (a < h ? 1 : sx) * (b < h ? 1 : sy);
                // class 2 takes class 1's vector at the swapped representative
                const double val = cd.cls == 2 ? v[ar * h + br] : v[br * h + ar];
                out[b * m + a] = 0.5 * sg * val;
            }
        double gsum = 0.0;
        for (int q = 0; q < M; ++q) {
            const double g = std::fmod((q + 1.0) * (q + 1.0) * kGoldenFrac, 1.0) - 0.5;
            gsum += g * out[q];
        }
        MLS_REQUIRE(cd.lam > 0, "create: Matern KL eigenvalue not positive (raise kl_quad or lower K)");
        const double scale = (gsum > 0 ? 1.0 : -1.0) * std::sqrt(w / cd.lam);
        for (int q = 0; q < M; ++q) out[q] *= scale;
        ctx->sqrt_lam[k] = std::sqrt(cd.lam);
    }
    TmpBuf dVs;
    MLS_TRY(dVs.b.ensure(sizeof(double) * Vs.size()));
    MLS_CHECK_HIP(hipMemcpy(dVs.b.ptr, Vs.data(), sizeof(double) * Vs.size(), hipMemcpyHostToDevice));
    const int Kp = (K + 31) / 32 * 32;
    for (int l = p.l_min; l <= p.l_max; ++l) {
        const int64_t ne = n_elem(l);
        MLS_CHECK_HIP(hipMalloc(&ctx->d_B[l], sizeof(double) * (size_t)K * ne));
        dim3 g((unsigned)((ne + 63) / 64), (unsigned)((K + 63) / 64));
        nystrom_extend_kernel<<<g, 256>>>(dVs.b.as<double>(), K, m, sc, p.sigma2, l, ctx->d_B[l]);
        MLS_CHECK_HIP(hipGetLastError());
        if (p.precision == MLS2MC_MIXED) {
            MLS_CHECK_HIP(hipMalloc(&ctx->d_B16[l], sizeof(__hip_bfloat16) * (size_t)Kp * ne));
            basis_to_bf16<<<(unsigned)((ne + 255) / 256), 256>>>(ctx->d_B[l], K, Kp, ne, ctx->d_B16[l]);
            MLS_CHECK_HIP(hipGetLastError());
        }
    }
    MLS_CHECK_HIP(hipDeviceSynchronize());
    return MLS2MC_OK;
}

}  // namespace mls
