// Batched forward solve of the P1 finite-element system of Sec. 5,
//   -div(kappa grad p) = 1 on (0,1)^2,  p = 0 on the boundary,
// on the uniform mesh with 2 n^2 right triangles (n = 2^l, diagonal from
// (i,j) to (i+1,j+1)), followed by the point observations (Sec. 2.1
// forward response operator, Sec. 5 observation operator).
//
// Design (gfx950): one persistent workgroup owns one particle at a time and
// runs its whole solve in a single launch; every global reduction of CG is
// a workgroup reduction, so there is no per-iteration kernel boundary and
// each particle stops at its own iteration count.  Workspaces are per
// workgroup slot (not per particle), so the footprint is independent of N.
//
// Discretisation facts used (derived from the P1 element matrices, checked
// by the tests against a generic assembly): every triangle is right-angled,
// the hypotenuse coupling vanishes, and the stiffness matrix is the 5-point
// operator (A x)_ij = sum over the four edges of w_e (x_ij - x_nb) with
// w_e = (kappa_T1 + kappa_T2)/2 over the two triangles having the edge as a
// leg.  The load for f = 1 is b_ij = h^2.
//
// Preconditioner: geometric multigrid V(1,1) cycle.  The coarse spaces are
// the nested P1 spaces of the coarser meshes (same diagonal direction), the
// prolongation is P1 interpolation and the restriction its transpose, and
// the Galerkin coarse operator P^T A P is exactly the P1 operator with the
// per-triangle coefficient averaged over the four children - again a
// 5-point operator.  Smoother: red-black Gauss-Seidel, red then black before
// the coarse correction and black then red after it, which makes the cycle
// a symmetric positive definite preconditioner.  Coarsest level l = 1 has one
// unknown and is solved exactly.
#include "common.h"

namespace mls {

// ------------------------------------------------------------ layout --
// Padded node grids (n+1)^2, node (i,j) at j(n+1)+i, boundary entries 0.
// wx[j][i]: weight of edge (i,j)-(i+1,j); wy[j][i]: edge (i,j)-(i,j+1).
// Slot layout (elements of T):
//   fine level l:   X R Z P Q WX WY RES              8 S_l
//   coarse L<l:     WX WY XC BC RESC                 5 S_L    then
//                   KAP (per-triangle kappa)         2 n_L^2
__host__ __device__ inline int64_t pad_sz(int L) { return ((int64_t(1) << L) + 1) * ((int64_t(1) << L) + 1); }
__host__ __device__ inline int64_t coarse_sz(int L) { return 5 * pad_sz(L) + 2 * (int64_t(1) << (2 * L)); }

__host__ __device__ inline int64_t coarse_off(int l, int L)
{
    int64_t o = 8 * pad_sz(l);
    for (int k = l - 1; k > L; --k) o += coarse_sz(k);
    return o;
}

__host__ __device__ inline int64_t slot_elems_hd(int l, bool mixed)
{
    int64_t o = 8 * pad_sz(l);
    for (int k = l - 1; k >= 1; --k) o += coarse_sz(k);
    if (mixed) o += 4 * pad_sz(l) + 2;  // float slot: + FP64 X64 and R64 (2 floats each)
    return o;
}

int64_t solver_slot_elems(int l, bool mixed) { return slot_elems_hd(l, mixed); }

template <typename T>
struct Lv {
    T *wx, *wy, *x, *b, *res, *kap;
    int n, lg, s;
};

template <typename T>
__device__ inline Lv<T> coarse_level(T* slot, int l, int L)
{
    Lv<T> v;
    T* base = slot + coarse_off(l, L);
    const int64_t S = pad_sz(L);
    v.wx = base; v.wy = base + S; v.x = base + 2 * S; v.b = base + 3 * S; v.res = base + 4 * S;
    v.kap = base + 5 * S;
    v.n = 1 << L; v.lg = L; v.s = v.n + 1;
    return v;
}

// ----------------------------------------------------------- stencils --
template <typename T>
__device__ __forceinline__ T diag_at(const T* __restrict__ wx, const T* __restrict__ wy, int c, int s)
{
    return wx[c - 1] + wx[c] + wy[c - s] + wy[c];
}

template <typename T>
__device__ __forceinline__ T nb_sum(const T* __restrict__ wx, const T* __restrict__ wy,
                                    const T* __restrict__ x, int c, int s)
{
    return wx[c - 1] * x[c - 1] + wx[c] * x[c + 1] + wy[c - s] * x[c - s] + wy[c] * x[c + s];
}

// loops over interior nodes: t in [0, (n-1) n), i = t mod n (skip 0)
#define MLS_FOR_INTERIOR(L, ...)                                                  \
    for (int t_ = threadIdx.x; t_ < (((L).n - 1) << (L).lg); t_ += BS) {            \
        const int i = t_ & ((L).n - 1);                                             \
        if (i == 0) continue;                                                       \
        const int j = 1 + (t_ >> (L).lg);                                           \
        const int c = j * (L).s + i;                                                \
        __VA_ARGS__                                                                 \
    }

// nodes of one colour: (i + j) mod 2 == col
#define MLS_FOR_COLOUR(L, col, ...)                                               \
    for (int t_ = threadIdx.x; t_ < (((L).n - 1) << ((L).lg - 1)); t_ += BS) {      \
        const int j = 1 + (t_ >> ((L).lg - 1));                                     \
        const int i = 2 * (t_ & (((L).n >> 1) - 1)) + 1 + (((col) + j + 1) & 1);   \
        if (i >= (L).n) continue;                                                   \
        const int c = j * (L).s + i;                                                \
        __VA_ARGS__                                                                 \
    }

template <int BS, typename T>
__device__ void zero_boundary(T* a, int n)
{
    const int s = n + 1;
    for (int t = threadIdx.x; t < 4 * s; t += BS) {
        const int k = t % s, side = t / s;
        int c = side == 0 ? k : side == 1 ? n * s + k : side == 2 ? k * s : k * s + n;
        a[c] = T(0);
    }
}

// edge weights of a level from its per-triangle coefficient; element
// 2(jn+i) is the lower, 2(jn+i)+1 the upper triangle of cell (i,j)
template <int BS, typename T, typename KT>
__device__ void edge_weights(const KT* __restrict__ kap, T* __restrict__ wx, T* __restrict__ wy,
                             int n, int lg)
{
    const int s = n + 1;
    for (int t = threadIdx.x; t < s * s; t += BS) {
        const int j = t / s, i = t - j * s;
        T vx = T(0), vy = T(0);
        if (i < n) {  // horizontal edge (i,j)-(i+1,j): lower of (i,j), upper of (i,j-1)
            double a = (j < n) ? (double)kap[2 * ((j << lg) + i)] : 0.0;
            double b = (j > 0) ? (double)kap[2 * (((j - 1) << lg) + i) + 1] : 0.0;
            vx = T(0.5 * (a + b));
        }
        if (j < n) {  // vertical edge (i,j)-(i,j+1): upper of (i,j), lower of (i-1,j)
            double a = (i < n) ? (double)kap[2 * ((j << lg) + i) + 1] : 0.0;
            double b = (i > 0) ? (double)kap[2 * ((j << lg) + i - 1)] : 0.0;
            vy = T(0.5 * (a + b));
        }
        wx[t] = vx;
        wy[t] = vy;
    }
}

// Galerkin coarsening of the per-triangle coefficient: each coarse
// triangle is the union of four fine ones (nested meshes, same diagonal).
template <int BS, typename KT, typename T>
__device__ void coarsen_kappa(const KT* __restrict__ kf, T* __restrict__ kc, int Lc)
{
    const int nc = 1 << Lc, lgf = Lc + 1;
    for (int t = threadIdx.x; t < nc * nc; t += BS) {
        const int I = t & (nc - 1), J = t >> Lc;
        const int i0 = 2 * I, j0 = 2 * J;
#define KF(ii, jj, tt) ((double)kf[2 * (((jj) << lgf) + (ii)) + (tt)])
        const double lo = 0.25 * (KF(i0, j0, 0) + KF(i0 + 1, j0, 0) + KF(i0 + 1, j0 + 1, 0) + KF(i0 + 1, j0, 1));
        const double up = 0.25 * (KF(i0, j0, 1) + KF(i0 + 1, j0 + 1, 1) + KF(i0, j0 + 1, 1) + KF(i0, j0 + 1, 0));
#undef KF
        kc[2 * t] = T(lo);
        kc[2 * t + 1] = T(up);
    }
}

// ------------------------------------------------------------ V-cycle --
template <int BS, typename T>
__device__ void smooth_colour(const Lv<T>& L, const T* __restrict__ b, T* __restrict__ x, int col,
                              bool first)
{
    if (first) {  // the other colour is still zero
        MLS_FOR_COLOUR(L, col, { x[c] = b[c] / diag_at(L.wx, L.wy, c, L.s); })
    } else {
        MLS_FOR_COLOUR(L, col, { x[c] = (b[c] + nb_sum(L.wx, L.wy, x, c, L.s)) / diag_at(L.wx, L.wy, c, L.s); })
    }
}

template <int BS, typename T>
__device__ void vcycle(T* slot, int l, const Lv<T>& F, const T* __restrict__ rhs, T* __restrict__ sol)
{
    if (l == 1) {  // the fine level is the coarsest: one unknown, exact
        if (threadIdx.x == 0) {
            const int c = F.s + 1;
            sol[c] = T((double)rhs[c] / (double)diag_at(F.wx, F.wy, c, F.s));
        }
        __syncthreads();
        return;
    }
    // down
    for (int Lk = l; Lk >= 2; --Lk) {
        const Lv<T> L = (Lk == l) ? F : coarse_level(slot, l, Lk);
        const T* b = (Lk == l) ? rhs : L.b;
        T* x = (Lk == l) ? sol : L.x;
        smooth_colour<BS>(L, b, x, 0, true);
        __syncthreads();
        smooth_colour<BS>(L, b, x, 1, false);
        __syncthreads();
        MLS_FOR_INTERIOR(L, {
            L.res[c] = b[c] - (diag_at(L.wx, L.wy, c, L.s) * x[c] - nb_sum(L.wx, L.wy, x, c, L.s));
        })
        __syncthreads();
        const Lv<T> C = coarse_level(slot, l, Lk - 1);
        const int s = L.s;
        const T* r = L.res;
        MLS_FOR_INTERIOR(C, {
            const int f = (2 * j) * s + 2 * i;
            C.b[c] = r[f] + T(0.5) * (r[f - 1] + r[f + 1] + r[f - s] + r[f + s] + r[f + s + 1] + r[f - s - 1]);
        })
        __syncthreads();
    }
    {  // coarsest level, one unknown at (1,1)
        const Lv<T> C = coarse_level(slot, l, 1);
        if (threadIdx.x == 0) {
            const int c = C.s + 1;  // solved in FP64 for either working type
            C.x[c] = T((double)C.b[c] / (double)diag_at(C.wx, C.wy, c, C.s));
        }
        __syncthreads();
    }
    // up
    for (int Lk = 2; Lk <= l; ++Lk) {
        const Lv<T> L = (Lk == l) ? F : coarse_level(slot, l, Lk);
        const Lv<T> C = coarse_level(slot, l, Lk - 1);
        const T* b = (Lk == l) ? rhs : L.b;
        T* x = (Lk == l) ? sol : L.x;
        const int sc = C.s;
        const T* xc = C.x;
        MLS_FOR_INTERIOR(L, {
            const int I = i >> 1, J = j >> 1;
            T v;
            if (!(i & 1) && !(j & 1)) v = xc[J * sc + I];
            else if ((i & 1) && !(j & 1)) v = T(0.5) * (xc[J * sc + I] + xc[J * sc + I + 1]);
            else if (!(i & 1) && (j & 1)) v = T(0.5) * (xc[J * sc + I] + xc[(J + 1) * sc + I]);
            else v = T(0.5) * (xc[J * sc + I] + xc[(J + 1) * sc + I + 1]);
            x[c] += v;
        })
        __syncthreads();
        smooth_colour<BS>(L, b, x, 1, false);
        __syncthreads();
        smooth_colour<BS>(L, b, x, 0, false);
        __syncthreads();
    }
}

// ------------------------------------------------------- setup & obs --
template <int BS, typename T, typename KT>
__device__ void setup_hierarchy(T* slot, int l, const Lv<T>& F, const KT* __restrict__ kap)
{
    edge_weights<BS>(kap, F.wx, F.wy, F.n, F.lg);
    if (l >= 2) {
        Lv<T> C = coarse_level(slot, l, l - 1);
        coarsen_kappa<BS>(kap, C.kap, l - 1);
        __syncthreads();
        for (int L = l - 1; L >= 1; --L) {
            Lv<T> V = coarse_level(slot, l, L);
            edge_weights<BS>(V.kap, V.wx, V.wy, V.n, V.lg);
            zero_boundary<BS>(V.x, V.n);
            if (L >= 2) coarsen_kappa<BS>(V.kap, coarse_level(slot, l, L - 1).kap, L - 1);
            __syncthreads();
        }
    }
}

struct SolveParams {
    int l;
    int64_t N;
    const int64_t* N_dev;
    const void* kappa;
    void* ws;
    int64_t slot_elems;
    double* G;
    double* p_out;
    int8_t* status;
    int32_t* iters;
    const double* y;
    double* phi;
    const int32_t* obs_idx;
    const double* obs_w;
    int nobs;
    double inv_sigma;
    double tol2;
    int max_iters;
};

template <int BS, typename T>
__device__ double observe_and_store(const SolveParams& P, int64_t q, const T* X, int n, double* red)
{
    double ph = 0.0;
    for (int o = threadIdx.x; o < P.nobs; o += BS) {
        double g = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) g += P.obs_w[3 * o + k] * (double)X[P.obs_idx[3 * o + k]];
        P.G[q * P.nobs + o] = g;
        if (P.y) {
            const double r = (P.y[o] - g) * P.inv_sigma;
            ph += r * r;
        }
    }
    if (P.p_out) {
        const int64_t M = (int64_t)(n - 1) * (n - 1);
        for (int64_t t = threadIdx.x; t < M; t += BS) {
            const int j = 1 + (int)(t / (n - 1)), i = 1 + (int)(t % (n - 1));
            P.p_out[q * M + t] = (double)X[j * (n + 1) + i];
        }
    }
    return P.y ? block_sum<BS>(ph, red) : 0.0;
}

// ------------------------------------------------------- FP64 kernel --
template <int BS>
__global__ __launch_bounds__(BS) void solve_f64_kernel(SolveParams P)
{
    __shared__ double red[BS / 64];
    const int l = P.l;
    double* slot = (double*)P.ws + (int64_t)blockIdx.x * P.slot_elems;
    const int64_t S = pad_sz(l);
    double *X = slot, *R = slot + S, *Z = slot + 2 * S, *Pv = slot + 3 * S, *Q = slot + 4 * S;
    Lv<double> F;
    F.wx = slot + 5 * S; F.wy = slot + 6 * S; F.res = slot + 7 * S;
    F.x = Z; F.b = R; F.kap = nullptr;
    F.n = 1 << l; F.lg = l; F.s = F.n + 1;
    const int ne = 2 << (2 * l);
    const double h2 = 1.0 / (double)(F.n * F.n);
    const int64_t NN = P.N_dev ? min(P.N, *P.N_dev) : P.N;

    for (int64_t q = blockIdx.x; q < NN; q += gridDim.x) {
        const double* kap = (const double*)P.kappa + q * ne;
        zero_boundary<BS>(X, F.n);
        zero_boundary<BS>(Z, F.n);
        zero_boundary<BS>(Pv, F.n);
        setup_hierarchy<BS>(slot, l, F, kap);
        MLS_FOR_INTERIOR(F, { X[c] = 0.0; R[c] = h2; })
        __syncthreads();
        vcycle<BS>(slot, l, F, R, Z);
        double rz = 0.0;
        MLS_FOR_INTERIOR(F, { rz += R[c] * Z[c]; Pv[c] = Z[c]; })
        rz = block_sum<BS>(rz, red);
        const double rz0 = rz;
        int it = 0;
        int8_t st = 1;
        if (!(rz0 > 0.0) || !isfinite(rz0)) st = 2;
        while (st == 1 && it < P.max_iters) {
            double pq = 0.0;
            MLS_FOR_INTERIOR(F, {
                const double v = diag_at(F.wx, F.wy, c, F.s) * Pv[c] - nb_sum(F.wx, F.wy, Pv, c, F.s);
                Q[c] = v;
                pq += Pv[c] * v;
            })
            pq = block_sum<BS>(pq, red);
            const double alpha = rz / pq;
            MLS_FOR_INTERIOR(F, {
                X[c] += alpha * Pv[c];
                R[c] -= alpha * Q[c];
            })
            __syncthreads();
            vcycle<BS>(slot, l, F, R, Z);
            double rzn = 0.0;
            MLS_FOR_INTERIOR(F, { rzn += R[c] * Z[c]; })
            rzn = block_sum<BS>(rzn, red);
            ++it;
            if (!isfinite(rzn)) { st = 2; break; }
            if (rzn <= P.tol2 * rz0) { st = 0; break; }
            const double beta = rzn / rz;
            rz = rzn;
            MLS_FOR_INTERIOR(F, { Pv[c] = Z[c] + beta * Pv[c]; })
            __syncthreads();
        }
        double ph = observe_and_store<BS>(P, q, X, F.n, red);
        if (threadIdx.x == 0) {
            if (P.status) P.status[q] = st;
            if (P.iters) P.iters[q] = it;
            if (P.phi) P.phi[q] = 0.5 * ph;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------- mixed kernel --
// FP32 multigrid-PCG inside FP64 iterative refinement: the system matrix is
// the one defined by the FP32 edge weights (promoted exactly to FP64 for the
// residual), r64 = b - A x64 in FP64, the correction A d = r64 is solved
// with FP32 MG-PCG to a loose tolerance, x64 += d.  The coarsest solve of
// the hierarchy is done in FP64.
template <int BS>
__global__ __launch_bounds__(BS) void solve_mixed_kernel(SolveParams P)
{
    __shared__ double red[BS / 64];
    const int l = P.l;
    float* slot = (float*)P.ws + (int64_t)blockIdx.x * P.slot_elems;
    const int64_t S = pad_sz(l);
    float *X = slot, *R = slot + S, *Z = slot + 2 * S, *Pv = slot + 3 * S, *Q = slot + 4 * S;
    Lv<float> F;
    F.wx = slot + 5 * S; F.wy = slot + 6 * S; F.res = slot + 7 * S;
    F.x = Z; F.b = R; F.kap = nullptr;
    F.n = 1 << l; F.lg = l; F.s = F.n + 1;
    // FP64 arrays after the float hierarchy (8-byte aligned: slot_elems even)
    const int64_t hier = slot_elems_hd(l, false);
    double* X64 = (double*)(slot + ((hier + 1) & ~int64_t(1)));
    double* R64 = X64 + S;
    const int ne = 2 << (2 * l);
    const double h2 = 1.0 / (double)(F.n * F.n);
    const float inner_tol2 = 1e-10f;  // inner relative reduction 1e-5 per sweep
    const int max_outer = 12;
    const int64_t NN = P.N_dev ? min(P.N, *P.N_dev) : P.N;

    for (int64_t q = blockIdx.x; q < NN; q += gridDim.x) {
        const float* kap = (const float*)P.kappa + q * ne;
        zero_boundary<BS>(X, F.n);
        zero_boundary<BS>(Z, F.n);
        zero_boundary<BS>(Pv, F.n);
        zero_boundary<BS>(X64, F.n);
        setup_hierarchy<BS>(slot, l, F, kap);
        MLS_FOR_INTERIOR(F, { X64[c] = 0.0; R64[c] = h2; })
        __syncthreads();
        double rr0 = 0.0;
        MLS_FOR_INTERIOR(F, { rr0 += h2 * h2; })
        rr0 = block_sum<BS>(rr0, red);
        int it = 0;
        int8_t st = 1;
        for (int outer = 0; outer < max_outer && st == 1; ++outer) {
            // inner FP32 PCG on A d = r64, d in X (float), zero start
            MLS_FOR_INTERIOR(F, { X[c] = 0.f; R[c] = (float)R64[c]; })
            __syncthreads();
            vcycle<BS>(slot, l, F, R, Z);
            double rz = 0.0;
            MLS_FOR_INTERIOR(F, { rz += (double)R[c] * (double)Z[c]; Pv[c] = Z[c]; })
            rz = block_sum<BS>(rz, red);
            const double rzi0 = rz;
            for (int k = 0; k < P.max_iters && rz > 0.0; ++k) {
                double pq = 0.0;
                MLS_FOR_INTERIOR(F, {
                    const float v = diag_at(F.wx, F.wy, c, F.s) * Pv[c] - nb_sum(F.wx, F.wy, Pv, c, F.s);
                    Q[c] = v;
                    pq += (double)Pv[c] * (double)v;
                })
                pq = block_sum<BS>(pq, red);
                const float alpha = (float)(rz / pq);
                MLS_FOR_INTERIOR(F, {
                    X[c] += alpha * Pv[c];
                    R[c] -= alpha * Q[c];
                })
                __syncthreads();
                vcycle<BS>(slot, l, F, R, Z);
                double rzn = 0.0;
                MLS_FOR_INTERIOR(F, { rzn += (double)R[c] * (double)Z[c]; })
                rzn = block_sum<BS>(rzn, red);
                ++it;
                if (!isfinite(rzn)) { st = 2; break; }
                if (rzn <= (double)inner_tol2 * rzi0) break;
                const float beta = (float)(rzn / rz);
                rz = rzn;
                MLS_FOR_INTERIOR(F, { Pv[c] = Z[c] + beta * Pv[c]; })
                __syncthreads();
            }
            if (st == 2) break;
            // x64 += d; r64 = b - A x64 in FP64 with the FP32 weights promoted
            MLS_FOR_INTERIOR(F, { X64[c] += (double)X[c]; })
            __syncthreads();
            double rr = 0.0;
            MLS_FOR_INTERIOR(F, {
                const double d = (double)F.wx[c - 1] + (double)F.wx[c] + (double)F.wy[c - F.s] + (double)F.wy[c];
                const double nb = (double)F.wx[c - 1] * X64[c - 1] + (double)F.wx[c] * X64[c + 1]
                                + (double)F.wy[c - F.s] * X64[c - F.s] + (double)F.wy[c] * X64[c + F.s];
                const double r = h2 - (d * X64[c] - nb);
                R64[c] = r;
                rr += r * r;
            })
            rr = block_sum<BS>(rr, red);
            if (!isfinite(rr)) { st = 2; break; }
            if (rr <= P.tol2 * rr0) st = 0;
        }
        double ph = observe_and_store<BS>(P, q, X64, F.n, red);
        if (threadIdx.x == 0) {
            if (P.status) P.status[q] = st;
            if (P.iters) P.iters[q] = it;
            if (P.phi) P.phi[q] = 0.5 * ph;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ launch --
static int default_block(int l)
{
    if (l <= 4) return 64;
    if (l == 5) return 128;
    if (l == 6) return 256;
    return 512;
}

int launch_solve(mls2mc_ctx* ctx, const SolveArgs& a, hipStream_t s)
{
    if (a.N == 0) return MLS2MC_OK;
    const int l = a.l;
    const bool mixed = a.kappa_f32;
    const int dev_cus = ctx->n_cu;
    int64_t slot = solver_slot_elems(l, mixed);
    slot = (slot + 63) & ~int64_t(63);  // 256/512-byte aligned slots
    const size_t esz = mixed ? sizeof(float) : sizeof(double);
    int bs = ctx->solver_block[l] ? ctx->solver_block[l] : default_block(l);
    int64_t grid = ctx->solver_grid[l] ? ctx->solver_grid[l] : (int64_t)dev_cus * (l <= 6 ? 8 : 4);
    // cap the slot workspace at 16 GiB
    const int64_t cap = (int64_t)((16ull << 30) / (slot * esz));
    if (grid > cap) grid = cap;
    if (grid > a.N) grid = a.N;
    if (grid < 1) grid = 1;
    MLS_TRY(ctx->ws_solver.ensure((size_t)grid * slot * esz));
    SolveParams P;
    P.l = l; P.N = a.N; P.N_dev = a.N_dev; P.kappa = a.kappa; P.ws = ctx->ws_solver.ptr; P.slot_elems = slot;
    P.G = a.G; P.p_out = a.p_out; P.status = a.status; P.iters = a.iters; P.y = a.y; P.phi = a.phi;
    P.obs_idx = ctx->obs[l].idx; P.obs_w = ctx->obs[l].w; P.nobs = ctx->nobs;
    P.inv_sigma = 1.0 / ctx->prob.sigma_n;
    P.tol2 = ctx->rtol * ctx->rtol;
    P.max_iters = ctx->max_iters;
    ProfRec rec;
    if (ctx->prof_on) {
        if (!P.iters) {  // the iteration totals need per-particle counts
            MLS_TRY(ctx->ws_prof.ensure(sizeof(int32_t) * (size_t)a.N));
            P.iters = ctx->ws_prof.as<int32_t>();
        }
        MLS_TRY(prof_begin(ctx, MLS2MC_PROF_SOLVE, l, a.N, s, &rec));
    }
    dim3 g((unsigned)grid);
#define MLS_LAUNCH(BSV)                                                              \
    if (mixed) solve_mixed_kernel<BSV><<<g, BSV, 0, s>>>(P);                         \
    else solve_f64_kernel<BSV><<<g, BSV, 0, s>>>(P);
    switch (bs) {
        case 64: MLS_LAUNCH(64) break;
        case 128: MLS_LAUNCH(128) break;
        case 256: MLS_LAUNCH(256) break;
        case 512: MLS_LAUNCH(512) break;
        case 1024: MLS_LAUNCH(1024) break;
        default: MLS_REQUIRE(false, "solver: unsupported block size");
    }
#undef MLS_LAUNCH
    MLS_CHECK_HIP(hipGetLastError());
    if (ctx->prof_on) {
        MLS_TRY(prof_end(ctx, MLS2MC_PROF_SOLVE, l, rec, s));
        MLS_TRY(launch_reduce_i32(a.N, P.iters, nullptr, ctx->d_prof_iters + 2 * l, s));
    }
    return MLS2MC_OK;
}

// ------------------------------------------------------ observations --
// P1 interpolation at (a/(m+1), b/(m+1)): cell i = min(floor(x n), n-1),
// local xi = x n - i; lower triangle if xi >= eta.
int build_obs_tables(mls2mc_ctx* ctx)
{
    const int m = ctx->prob.m;
    const int nobs = m * m;
    ctx->nobs = nobs;
    for (int l = ctx->prob.l_min; l <= ctx->prob.l_max; ++l) {
        const int n = 1 << l, s = n + 1;
        std::vector<int32_t> idx(3 * nobs);
        std::vector<double> w(3 * nobs);
        for (int bb = 1; bb <= m; ++bb)
            for (int aa = 1; aa <= m; ++aa) {
                const int o = (bb - 1) * m + (aa - 1);
                const double x = (double)aa / (double)(m + 1), y = (double)bb / (double)(m + 1);
                int i = (int)std::floor(x * n), j = (int)std::floor(y * n);
                if (i > n - 1) i = n - 1;
                if (j > n - 1) j = n - 1;
                const double xi = x * n - i, eta = y * n - j;
                int nodes[3];
                double wt[3];
                nodes[0] = j * s + i;
                if (xi >= eta) {
                    nodes[1] = j * s + i + 1; nodes[2] = (j + 1) * s + i + 1;
                    wt[0] = 1.0 - xi; wt[1] = xi - eta; wt[2] = eta;
                } else {
                    nodes[1] = (j + 1) * s + i + 1; nodes[2] = (j + 1) * s + i;
                    wt[0] = 1.0 - eta; wt[1] = xi; wt[2] = eta - xi;
                }
                for (int k = 0; k < 3; ++k) { idx[3 * o + k] = nodes[k]; w[3 * o + k] = wt[k]; }
            }
        MLS_CHECK_HIP(hipMalloc(&ctx->obs[l].idx, sizeof(int32_t) * idx.size()));
        MLS_CHECK_HIP(hipMalloc(&ctx->obs[l].w, sizeof(double) * w.size()));
        MLS_CHECK_HIP(hipMemcpy(ctx->obs[l].idx, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice));
        MLS_CHECK_HIP(hipMemcpy(ctx->obs[l].w, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice));
    }
    return MLS2MC_OK;
}

}  // namespace mls
