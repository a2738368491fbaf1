// Flow-cell forward problem (Sec. 5, Example 5.3): P1 finite elements for
//   -div(kappa grad p) = 0 on (0,1)^2,  p = 0 on x1 = 0,  p = 1 on x1 = 1,
//   no flow through x2 = 0 and x2 = 1,
// solved by multigrid-preconditioned CG with one persistent workgroup per
// particle, like the Dirichlet solver, on a layout of its own.
//
// Layout of level L (n = 2^L): nodes (i, j), 0 <= i <= n, with a ghost row
// below j = 0 and above j = n; index c = (j + 1)(n + 1) + i, (n+1)(n+3)
// entries.  Unknowns are 1 <= i <= n-1, 0 <= j <= n (the two no-flow rows
// included), u = j (n-1) + (i-1).  The operator is the 5-point form of P1 on
// the SW-NE mesh: the weight of an edge is half the sum of the coefficients
// of the (one or two) triangles that have it as a leg, so the no-flow rows get
// their natural one-sided weights and the edges to the ghost rows weigh 0.
// The Dirichlet value 1 at i = n enters the right-hand side through the
// weights of the edges (n-1, j)-(n, j); the iterates hold 0 on both
// Dirichlet columns.
//
// V-cycle: red-black Gauss-Seidel (red first down, black first up, so the
// cycle is symmetric), restriction by the transpose of P1 interpolation,
// coarse coefficients averaged over the four children of each coarse
// triangle (the Galerkin operator of the nested meshes), an exact
// tridiagonal solve at h = 1/2 (three unknowns on the column i = 1).
//
// Fused passes: p = z + beta p_old is formed inside the operator apply
// (double-buffered p); the x/r update also does the V-cycle's first red
// sweep from z = 0; the residual, which after a black sweep lives on the red
// nodes only, is formed inside the restriction, which also does the coarse
// level's first red sweep; <r, z> is summed in the last red sweep.
#include "common.h"

namespace mls {

namespace {

__host__ __device__ inline int64_t fsz(int L)
{
    const int64_t n = int64_t(1) << L;
    return (n + 1) * (n + 3);
}

// slot: fine arrays, then per coarse level l-1 .. 1 its arrays and coefficients.
// F_W32 holds the FP32-rounded fine weights WX then WY (2 fsz floats): the
// V-cycle's fine level reads those, while the CG operator keeps the FP64
// ones, so the preconditioner is a fixed SPD operator close to A that reads
// half the weight bytes.
enum { F_U = 0, F_R, F_Z, F_P, F_P2, F_Q, F_WX, F_WY, F_W32, F_COUNT };
enum { C_X = 0, C_B, C_WX, C_WY, C_COUNT };

__host__ __device__ inline int64_t coarse_base(int l, int L)
{
    int64_t o = F_COUNT * fsz(l);
    for (int k = l - 1; k > L; --k) o += C_COUNT * fsz(k) + (int64_t(2) << (2 * k));
    return o;
}

__host__ __device__ inline int64_t flow_slot(int l) { return coarse_base(l, 0); }

// Coarse levels 1 .. ltop keep X, B, WX and WY in LDS (level 1 first, in
// elements of double); their coefficients stay in the slot.
__host__ __device__ inline int64_t flow_lds_off(int L)
{
    int64_t o = 0;
    for (int k = 1; k < L; ++k) o += C_COUNT * fsz(k);
    return o;
}

// the finest coarse level whose hierarchy fits the budget (0: none)
inline int flow_lds_top(int l, int64_t budget_bytes)
{
    int top = 0;
    for (int L = 1; L < l; ++L)
        if (flow_lds_off(L + 1) * (int64_t)sizeof(double) <= budget_bytes) top = L;
    return top;
}

// where a particle's arrays live: its slot, and the LDS levels
struct FSlot {
    double* slot;
    double* lds;
    int ltop;
};

template <typename W>
struct FLvT {
    double *x, *b;
    W *wx, *wy;  // edge weights, promoted exactly to FP64 where used
    double* kc;
    int n, s;
};
using FLv = FLvT<double>;

// level L of the hierarchy of the slot (L = l: the fine level's V-cycle
// arrays, x = Z, b = R)
__device__ inline FLv flevel(const FSlot& S, int l, int L)
{
    double* slot = S.slot;
    FLv v;
    v.n = 1 << L;
    v.s = v.n + 1;
    const int64_t f = fsz(L);
    if (L == l) {
        v.x = slot + F_Z * f;
        v.b = slot + F_R * f;
        v.wx = slot + F_WX * f;
        v.wy = slot + F_WY * f;
        v.kc = nullptr;
    } else {
        double* g = slot + coarse_base(l, L);
        double* base = L <= S.ltop ? S.lds + flow_lds_off(L) : g;
        v.x = base + C_X * f;
        v.b = base + C_B * f;
        v.wx = base + C_WX * f;
        v.wy = base + C_WY * f;
        v.kc = g + C_COUNT * f;
    }
    return v;
}

// the fine level as the V-cycle sees it: x = Z, b = R, FP32 weights
__device__ inline FLvT<float> flevel32(double* slot, int l)
{
    FLvT<float> v;
    v.n = 1 << l;
    v.s = v.n + 1;
    const int64_t f = fsz(l);
    v.x = slot + F_Z * f;
    v.b = slot + F_R * f;
    v.wx = reinterpret_cast<float*>(slot + F_W32 * f);
    v.wy = v.wx + f;
    v.kc = nullptr;
    return v;
}

#define FLOW_FOR_UNK(n_, ...)                                                  \
    for (int t_ = threadIdx.x; t_ < ((n_) - 1) * ((n_) + 1); t_ += BS) {     \
        const int i = 1 + t_ % ((n_) - 1), j = t_ / ((n_) - 1);              \
        const int c = (j + 1) * ((n_) + 1) + i;                              \
        __VA_ARGS__                                                          \
    }

template <typename W>
__device__ __forceinline__ double fdiag(const FLvT<W>& L, int c)
{
    return (double)L.wx[c - 1] + (double)L.wx[c] + (double)L.wy[c - L.s] + (double)L.wy[c];
}

template <typename W>
__device__ __forceinline__ double fnb(const FLvT<W>& L, const double* x, int c)
{
    return (double)L.wx[c - 1] * x[c - 1] + (double)L.wx[c] * x[c + 1] + (double)L.wy[c - L.s] * x[c - L.s]
         + (double)L.wy[c] * x[c + L.s];
}

template <int BS>
__device__ void zero_all(double* a, int64_t n)
{
    for (int64_t t = threadIdx.x; t < n; t += BS) a[t] = 0.0;
}

// edge weights of a level from its element coefficients (kl: lower
// triangles at 2(jn+i), upper at 2(jn+i)+1)
template <int BS, typename KT>
__device__ void flow_weights(const FLv& L, const KT* __restrict__ ke, float* __restrict__ wx32 = nullptr,
                             float* __restrict__ wy32 = nullptr)
{
    const int n = L.n, s = L.s;
    const int64_t tot = fsz(31 - __builtin_clz(n));
    for (int64_t c = threadIdx.x; c < tot; c += BS) {
        const int i = (int)(c % s), j = (int)(c / s) - 1;
        double wxv = 0.0, wyv = 0.0;
        if (i < n && j >= 0 && j <= n) {  // edge (i,j)-(i+1,j)
            const double lo = j < n ? (double)ke[2 * (j * n + i)] : 0.0;
            const double up = j > 0 ? (double)ke[2 * ((j - 1) * n + i) + 1] : 0.0;
            wxv = 0.5 * (lo + up);
        }
        if (j >= 0 && j < n) {  // edge (i,j)-(i,j+1)
            const double lo = i > 0 ? (double)ke[2 * (j * n + i - 1)] : 0.0;
            const double up = i < n ? (double)ke[2 * (j * n + i) + 1] : 0.0;
            wyv = 0.5 * (lo + up);
        }
        L.wx[c] = wxv;
        L.wy[c] = wyv;
        if (wx32) {  // FP32-rounded copies for the V-cycle
            wx32[c] = (float)wxv;
            wy32[c] = (float)wyv;
        }
    }
}

// coefficients of level Lc = Lf - 1: each coarse triangle averages its four children
template <int BS, typename KT>
__device__ void flow_coarsen(const KT* __restrict__ kf, double* __restrict__ kc, int nc)
{
    const int nf = 2 * nc;
    for (int t = threadIdx.x; t < nc * nc; t += BS) {
        const int I = t % nc, J = t / nc;
        auto lo = [&](int i, int j) { return (double)kf[2 * (j * nf + i)]; };
        auto up = [&](int i, int j) { return (double)kf[2 * (j * nf + i) + 1]; };
        const int i0 = 2 * I, j0 = 2 * J;
        kc[2 * t] = 0.25 * (lo(i0, j0) + lo(i0 + 1, j0) + lo(i0 + 1, j0 + 1) + up(i0 + 1, j0));
        kc[2 * t + 1] = 0.25 * (up(i0, j0) + up(i0, j0 + 1) + up(i0 + 1, j0 + 1) + lo(i0, j0 + 1));
    }
}

template <int BS, typename W>
__device__ void smooth(const FLvT<W>& L, int col)
{
    FLOW_FOR_UNK(L.n, {
        if (((i + j) & 1) != col) continue;
        L.x[c] = (L.b[c] + fnb(L, L.x, c)) / fdiag(L, c);
    })
    __syncthreads();
}

// residual b - A x at an unknown node f
template <typename W>
__device__ __forceinline__ double fres(const FLvT<W>& F, int f)
{
    return F.b[f] - (fdiag(F, f) * F.x[f] - fnb(F, F.x, f));
}

// ends a red sweep with sum_c b_c x_c over the unknowns (x final everywhere)
template <int BS, typename W>
__device__ double smooth_red_dot(const FLvT<W>& L, double* red)
{
    double d = 0.0;
    FLOW_FOR_UNK(L.n, {
        double x = L.x[c];
        if (!((i + j) & 1)) {
            x = (L.b[c] + fnb(L, L.x, c)) / fdiag(L, c);
            L.x[c] = x;
        }
        d += L.b[c] * x;
    })
    return block_sum<BS>(d, red);
}

// C.b = P^T (F.b - A F.x) right after a black sweep: the black residuals
// vanish, so the coarse node (I, J) gathers the red residuals at (2I, 2J),
// (2I+1, 2J+1) and (2I-1, 2J-1).  C.x gets the coarse first red sweep from 0.
template <int BS, typename W>
__device__ void restrict_red(const FLvT<W>& F, const FLv& C)
{
    const int fs = F.s, nf = F.n;
    FLOW_FOR_UNK(C.n, {
        const int f = (2 * j + 1) * fs + 2 * i;
        double v = fres(F, f);
        if (2 * j + 1 <= nf) v += 0.5 * fres(F, f + fs + 1);
        if (j >= 1) v += 0.5 * fres(F, f - fs - 1);
        C.b[c] = v;
        C.x[c] = ((i + j) & 1) ? 0.0 : v / fdiag(C, c);
    })
    __syncthreads();
}

// F.x += P C.x
template <int BS, typename W>
__device__ void prolong_add(const FLv& C, const FLvT<W>& F)
{
    const int cs = C.s;
    FLOW_FOR_UNK(F.n, {
        const int I = i >> 1, Jc = j >> 1;
        const int q = (Jc + 1) * cs + I;
        double v;
        if (!(i & 1) && !(j & 1)) v = C.x[q];
        else if ((i & 1) && !(j & 1)) v = 0.5 * (C.x[q] + C.x[q + 1]);
        else if (!(i & 1)) v = 0.5 * (C.x[q] + C.x[q + cs]);
        else v = 0.5 * (C.x[q] + C.x[q + cs + 1]);
        F.x[c] += v;
    })
    __syncthreads();
}

// The first black sweep of the up-leg with the coarse correction x += P e
// folded in.  A black node's four neighbours are red, and their corrected
// values are read only by this sweep (the red sweep after it recomputes
// them), so the correction is interpolated at the neighbours on the fly and
// never stored; the black nodes' own corrections would be overwritten.  As
// in prolong_add, only unknown nodes take a correction; a red unknown has
// both indices even (a coarse node) or both odd (the middle of a coarse
// diagonal edge).
template <int BS, typename W>
__device__ void smooth_black_corrected(const FLvT<W>& L, const FLv& C)
{
    const int n = L.n, s = L.s, cs = C.s;
    auto pe = [&](int i, int j) -> double {
        if (i < 1 || i > n - 1 || j < 0 || j > n) return 0.0;
        const int q = ((j >> 1) + 1) * cs + (i >> 1);
        return (i & 1) ? 0.5 * (C.x[q] + C.x[q + cs + 1]) : C.x[q];
    };
    FLOW_FOR_UNK(n, {
        if (!((i + j) & 1)) continue;
        const double nb = (double)L.wx[c - 1] * (L.x[c - 1] + pe(i - 1, j))
                        + (double)L.wx[c] * (L.x[c + 1] + pe(i + 1, j))
                        + (double)L.wy[c - s] * (L.x[c - s] + pe(i, j - 1))
                        + (double)L.wy[c] * (L.x[c + s] + pe(i, j + 1));
        L.x[c] = (L.b[c] + nb) / fdiag(L, c);
    })
    __syncthreads();
}

// exact solve at h = 1/2: unknowns (1,0), (1,1), (1,2), a tridiagonal system
template <int BS>
__device__ void coarsest(const FLv& L)
{
    if (threadIdx.x == 0) {
        const int s = L.s, c0 = s + 1, c1 = 2 * s + 1, c2 = 3 * s + 1;
        const double d0 = fdiag(L, c0), d1 = fdiag(L, c1), d2 = fdiag(L, c2);
        const double e0 = L.wy[c0], e1 = L.wy[c1];
        // forward elimination of -e x_{k-1} + d x_k - e' x_{k+1} = b_k
        const double g0 = d0, y0 = L.b[c0];
        const double g1 = d1 - e0 * e0 / g0, y1 = L.b[c1] + e0 * y0 / g0;
        const double g2 = d2 - e1 * e1 / g1, y2 = L.b[c2] + e1 * y1 / g1;
        const double x2 = y2 / g2;
        const double x1 = (y1 + e1 * x2) / g1;
        const double x0 = (y0 + e0 * x1) / g0;
        L.x[c0] = x0;
        L.x[c1] = x1;
        L.x[c2] = x2;
    }
    __syncthreads();
}

constexpr int kFoldFrom = 7;  // levels that fold the coarse correction into the black sweep

// z = V r on the fine level l whose first red sweep (from z = 0) is done;
// returns <r, z>
template <int BS>
__device__ __forceinline__ double flow_vcycle(const FSlot& S, int l, int nu, double* red)
{
    if (l == 1) {  // the fine level is the coarsest: exact, FP64 weights
        const FLv F = flevel(S, l, l);
        coarsest<BS>(F);
        double d = 0.0;
        FLOW_FOR_UNK(F.n, { d += F.b[c] * F.x[c]; })
        return block_sum<BS>(d, red);
    }
    const FLvT<float> F32 = flevel32(S.slot, l);
    smooth<BS>(F32, 1);
    for (int k = 1; k < nu; ++k) {
        smooth<BS>(F32, 0);
        smooth<BS>(F32, 1);
    }
    restrict_red<BS>(F32, flevel(S, l, l - 1));
    for (int L = l - 1; L >= 2; --L) {
        const FLv V = flevel(S, l, L);
        smooth<BS>(V, 1);
        for (int k = 1; k < nu; ++k) {
            smooth<BS>(V, 0);
            smooth<BS>(V, 1);
        }
        restrict_red<BS>(V, flevel(S, l, L - 1));
    }
    coarsest<BS>(flevel(S, l, 1));
    // the coarse correction: folded into the first black sweep from h = 1/128
    // on (bitwise the same values); on the smaller levels the separate pass
    // measured faster than the on-the-fly interpolation
    for (int L = 2; L <= l - 1; ++L) {
        const FLv V = flevel(S, l, L);
        if (L < kFoldFrom) prolong_add<BS>(flevel(S, l, L - 1), V);
        for (int k = 0; k < nu; ++k) {
            if (k == 0 && L >= kFoldFrom) smooth_black_corrected<BS>(V, flevel(S, l, L - 1));
            else smooth<BS>(V, 1);
            smooth<BS>(V, 0);
        }
    }
    if (l < kFoldFrom) prolong_add<BS>(flevel(S, l, l - 1), F32);
    double dot = 0.0;
    for (int k = 0; k < nu; ++k) {
        if (k == 0 && l >= kFoldFrom) smooth_black_corrected<BS>(F32, flevel(S, l, l - 1));
        else smooth<BS>(F32, 1);
        if (k == nu - 1) dot = smooth_red_dot<BS>(F32, red);
        else smooth<BS>(F32, 0);
    }
    return dot;
}

struct FlowParams {
    int l;
    int64_t N;
    const int64_t* N_dev;
    const double* kappa;  // N x n_e
    double* ws;
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
    double inv_sigma, tol2;
    int max_iters, nu;
    int ltop;  // coarse levels 1 .. ltop in LDS
};

extern __shared__ __align__(16) double flow_lds[];

// The CG stencil pass by columns, for blocks that the row width n divides
// (BS = m n, from h = 1/64 on): the m groups of n threads take m bands of the
// n + 1 unknown rows, and thread i of a group owns column i of its band,
// keeping p and WY of the row below and of its own row in registers, so
// each row of Z, P_old and WY is loaded once per pass rather than three
// times.  Lane 0 of a group owns the Dirichlet column x1 = 0 and idles; the
// ghost rows below and above carry zero weights, as in the row loop.
__device__ __forceinline__ int flow_opaque(int c)  // keeps one 32-bit offset for all arrays
{
    asm("" : "+v"(c));
    return c;
}

template <int BS>
__device__ double flow_walk_apply(const FLv& F, const double* __restrict__ Z, const double* __restrict__ Po,
                                  double beta, double* __restrict__ Pn, double* __restrict__ Q)
{
    const int n = F.n, s = F.s, m = BS / n;
    const int i = threadIdx.x & (n - 1), band = threadIdx.x / n;
    const int rows = (n + m) / m;  // ceil((n + 1) / m)
    const int j0 = band * rows, j1 = min(n + 1, j0 + rows);
    double pq = 0.0;
    if (i == 0 || j0 >= j1) return pq;
    auto pn = [&](int q) { return Z[q] + beta * Po[q]; };
    const int c0 = j0 * s + i;  // the row below unknown row j0
    double pm = pn(c0), p0 = pn(c0 + s), wym = F.wy[c0];
#pragma unroll 1
    for (int j = j0; j < j1; ++j) {
        const int c = flow_opaque((j + 1) * s + i);
        const double pp = pn(c + s), wyc = F.wy[c];
        const double nb = F.wx[c - 1] * pn(c - 1) + F.wx[c] * pn(c + 1) + wym * pm + wyc * pp;
        const double qv = (F.wx[c - 1] + F.wx[c] + wym + wyc) * p0 - nb;
        Pn[c] = p0;
        Q[c] = qv;
        pq += p0 * qv;
        pm = p0;
        p0 = pp;
        wym = wyc;
    }
    return pq;
}

// PX: the launch returns the pressure field (p_out), so the iterate U is
// kept.  Without it the observations are gathered step by step: G = Obs U
// with U = the lifted boundary values + sum_k alpha_k p_k, so G starts at
// the observations of the lift and each step adds alpha_k Obs p_k, and the
// update pass neither reads nor writes U (16 B less per unknown and
// iteration).  Separate instances keep each variant's registers.
template <int BS, bool WK, bool PX>
__global__ __launch_bounds__(BS) void flow_solve_kernel(FlowParams P)
{
    __shared__ double red[BS / 64];
    const int l = P.l, n = 1 << l, s = n + 1;
    const int64_t ne = int64_t(2) << (2 * l), f = fsz(l);
    const int64_t NN = P.N_dev ? min(P.N, *P.N_dev) : P.N;
    double* slot = P.ws + (int64_t)blockIdx.x * P.slot_elems;
    double* U = slot + F_U * f;
    double* R = slot + F_R * f;
    double* Z = slot + F_Z * f;
    double* Q = slot + F_Q * f;
    const FSlot S{slot, flow_lds, P.ltop};
    const FLv F = flevel(S, l, l);
    const FLvT<float> F32 = flevel32(slot, l);  // the V-cycle's view of the fine level
    for (int64_t q = blockIdx.x; q < NN; q += gridDim.x) {
        const double* kap = P.kappa + q * ne;
        // set-up: zero the arrays, weights of every level, the lifted right-hand side
        zero_all<BS>(slot, F_COUNT * f);
        for (int L = l - 1; L >= 1; --L) zero_all<BS>(flevel(S, l, L).x, C_COUNT * fsz(L));
        __syncthreads();
        flow_weights<BS>(F, kap, F32.wx, F32.wy);
        if (l >= 2) flow_coarsen<BS>(kap, flevel(S, l, l - 1).kc, n / 2);
        __syncthreads();
        for (int L = l - 1; L >= 1; --L) {
            const FLv C = flevel(S, l, L);
            flow_weights<BS>(C, C.kc);
            if (L >= 2) flow_coarsen<BS>(C.kc, flevel(S, l, L - 1).kc, C.n / 2);
            __syncthreads();
        }
        // lifted right-hand side; z starts with the V-cycle's first red sweep;
        // the Dirichlet column i = n of U holds 1 (no step changes it)
        FLOW_FOR_UNK(n, {
            const double r = i == n - 1 ? F.wx[c] : 0.0;
            R[c] = r;
            Z[c] = ((i + j) & 1) ? 0.0 : r / fdiag(F32, c);
        })
        for (int j = threadIdx.x; j <= n; j += BS) U[(j + 1) * s + n] = 1.0;
        __syncthreads();
        double* Gq = P.G + q * P.nobs;
        if (!PX)  // the observations of the lift; thread o owns observation o
            for (int o = threadIdx.x; o < P.nobs; o += BS) {
                double g = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) g += P.obs_w[3 * o + k] * U[P.obs_idx[3 * o + k]];
                Gq[o] = g;
            }
        // PCG
        double rz = flow_vcycle<BS>(S, l, P.nu, red);
        const double rz0 = rz;
        double beta = 0.0;
        double* Po = slot + F_P * f;
        double* Pn = slot + F_P2 * f;
        int8_t st = 1;
        int it = 0;
        if (!(rz0 > 0.0)) st = isfinite(rz0) ? 0 : 2;
        while (st == 1 && it < P.max_iters) {
            ++it;
            // p = z + beta p_old and q = A p in one pass
            double pq = 0.0;
            if (WK && BS % n == 0) {
                pq = flow_walk_apply<BS>(F, Z, Po, beta, Pn, Q);
            } else {
                FLOW_FOR_UNK(n, {
                    const double pc = Z[c] + beta * Po[c];
                    const double nb = F.wx[c - 1] * (Z[c - 1] + beta * Po[c - 1]) +
                                      F.wx[c] * (Z[c + 1] + beta * Po[c + 1]) +
                                      F.wy[c - s] * (Z[c - s] + beta * Po[c - s]) +
                                      F.wy[c] * (Z[c + s] + beta * Po[c + s]);
                    const double qv = fdiag(F, c) * pc - nb;
                    Pn[c] = pc;
                    Q[c] = qv;
                    pq += pc * qv;
                })
            }
            pq = block_sum<BS>(pq, red);
            const double alpha = rz / pq;
            if (!PX)  // Pn is complete (the reduction's barriers)
                for (int o = threadIdx.x; o < P.nobs; o += BS) {
                    double g = 0.0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) g += P.obs_w[3 * o + k] * Pn[P.obs_idx[3 * o + k]];
                    Gq[o] += alpha * g;
                }
            FLOW_FOR_UNK(n, {
                if (PX) U[c] += alpha * Pn[c];
                const double r = R[c] - alpha * Q[c];
                R[c] = r;
                Z[c] = ((i + j) & 1) ? 0.0 : r / fdiag(F32, c);
            })
            __syncthreads();
            const double rzn = flow_vcycle<BS>(S, l, P.nu, red);
            if (!isfinite(rzn) || !isfinite(alpha)) { st = 2; break; }
            if (rzn <= P.tol2 * rz0) { st = 0; break; }
            beta = rzn / rz;
            rz = rzn;
            double* t = Po;
            Po = Pn;
            Pn = t;
        }
        // observe and store
        __syncthreads();
        double ph = 0.0;
        for (int o = threadIdx.x; o < P.nobs; o += BS) {
            double g = 0.0;
            if (PX) {
#pragma unroll
                for (int k = 0; k < 3; ++k) g += P.obs_w[3 * o + k] * U[P.obs_idx[3 * o + k]];
                Gq[o] = g;
            } else {
                g = Gq[o];
            }
            if (P.y) {
                const double r = (P.y[o] - g) * P.inv_sigma;
                ph += r * r;
            }
        }
        if (PX && P.p_out) {
            double* po = P.p_out + q * (int64_t)(n - 1) * (n + 1);
            FLOW_FOR_UNK(n, { po[t_] = U[c]; })
        }
        if (P.y) ph = block_sum<BS>(ph, red);
        if (threadIdx.x == 0) {
            if (P.status) P.status[q] = st;
            if (P.iters) P.iters[q] = it;
            if (P.phi) P.phi[q] = 0.5 * ph;
        }
        __syncthreads();
    }
}

}  // namespace

int64_t flow_unknowns(int l) { return ((int64_t(1) << l) - 1) * ((int64_t(1) << l) + 1); }

#define FLOW_SWITCH(bs, walk, PX, grid, lds, stream, params)                                       \
    switch (bs) {                                                                                \
        case 64: flow_solve_kernel<64, false, PX><<<grid, 64, lds, stream>>>(params); break;      \
        case 128: flow_solve_kernel<128, false, PX><<<grid, 128, lds, stream>>>(params); break;   \
        case 256:                                                                                \
            if (walk) flow_solve_kernel<256, true, PX><<<grid, 256, lds, stream>>>(params);       \
            else flow_solve_kernel<256, false, PX><<<grid, 256, lds, stream>>>(params);           \
            break;                                                                               \
        case 512:                                                                                \
            if (walk) flow_solve_kernel<512, true, PX><<<grid, 512, lds, stream>>>(params);       \
            else flow_solve_kernel<512, false, PX><<<grid, 512, lds, stream>>>(params);           \
            break;                                                                               \
        case 1024:                                                                               \
            if (walk) flow_solve_kernel<1024, true, PX><<<grid, 1024, lds, stream>>>(params);     \
            else flow_solve_kernel<1024, false, PX><<<grid, 1024, lds, stream>>>(params);         \
            break;                                                                               \
        default: MLS_REQUIRE(false, "flow cell: unsupported block size");                        \
    }

int launch_flow_solve(mls2mc_ctx* ctx, const SolveArgs& a, hipStream_t s)
{
    if (a.N == 0) return MLS2MC_OK;
    MLS_REQUIRE(!a.kappa_f32, "flow cell: FP64 coefficients only");
    const int l = a.l;
    int64_t slot = flow_slot(l);
    slot = (slot + 31) & ~int64_t(31);
    int bs = ctx->solver_block[l] ? ctx->solver_block[l] : (l <= 5 ? 256 : (l == 6 ? 512 : 1024));
    int64_t grid = ctx->solver_grid[l] ? ctx->solver_grid[l] : (int64_t)ctx->n_cu * 4;
    const int64_t cap = (int64_t)((16ull << 30) / (slot * sizeof(double)));
    if (grid > cap) grid = cap;
    if (grid > a.N) grid = a.N;
    if (grid < 1) grid = 1;
    MLS_TRY(ctx->ws_solver.ensure((size_t)grid * slot * sizeof(double)));
    FlowParams P;
    P.l = l; P.N = a.N; P.N_dev = a.N_dev; P.kappa = (const double*)a.kappa;
    P.ws = ctx->ws_solver.as<double>(); P.slot_elems = slot;
    P.G = a.G; P.p_out = a.p_out; P.status = a.status; P.iters = a.iters; P.y = a.y; P.phi = a.phi;
    P.obs_idx = ctx->obs[l].idx; P.obs_w = ctx->obs[l].w; P.nobs = ctx->nobs;
    P.inv_sigma = 1.0 / ctx->prob.sigma_n;
    P.tol2 = ctx->rtol * ctx->rtol;
    P.max_iters = ctx->max_iters;
    P.nu = ctx->solver_nu[l] > 0 ? ctx->solver_nu[l] : 1;
    // the level's LDS budget, as for the Dirichlet solver (0 = 64 KiB, -1 = none)
    int64_t budget = ctx->solver_lds[l] >= 0 ? (ctx->solver_lds[l] ? ctx->solver_lds[l] : 65536) : 0;
    if (budget > ctx->max_lds) budget = ctx->max_lds;
    P.ltop = flow_lds_top(l, budget);
    const size_t lds = (size_t)flow_lds_off(P.ltop + 1) * sizeof(double);
    ProfRec rec;
    if (ctx->prof_on) {
        if (!P.iters) {
            MLS_TRY(ctx->ws_prof.ensure(sizeof(int32_t) * (size_t)a.N));
            P.iters = ctx->ws_prof.as<int32_t>();
        }
        MLS_TRY(prof_begin(ctx, MLS2MC_PROF_SOLVE, l, a.N, s, &rec));
    }
    dim3 g((unsigned)grid);
    // the column walk of the stencil pass from h = 1/64 on, where the row
    // width divides the block (separate instances, so the others keep their
    // registers)
    const bool walk = l >= 6 && bs % (1 << l) == 0;
    if (P.p_out) {
        FLOW_SWITCH(bs, walk, true, g, lds, s, P)
    } else {
        FLOW_SWITCH(bs, walk, false, g, lds, s, P)
    }
    MLS_CHECK_HIP(hipGetLastError());
    if (ctx->prof_on) {
        MLS_TRY(prof_end(ctx, MLS2MC_PROF_SOLVE, l, rec, s));
        MLS_TRY(launch_reduce_i32(a.N, P.iters, nullptr, ctx->d_prof_iters + 2 * l, s));
    }
    return MLS2MC_OK;
}

}  // namespace mls
