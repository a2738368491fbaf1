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
#include <algorithm>
#include <type_traits>

#include "common.h"

namespace mls {

// ------------------------------------------------------------ layout --
// Padded node grids (n+1)^2, node (i,j) at j(n+1)+i, boundary entries 0.
// wx[j][i]: weight of edge (i,j)-(i+1,j); wy[j][i]: edge (i,j)-(i,j+1).
// Slot layout (elements of T):
//   fine level l:   X R Z P Q WX WY P2               8 S_l
//                   FP64 solver only: FP32 copies of WX WY for the
//                   V-cycle                          2 ceil(S_l / 2)
//   coarse L<l:     WX WY XC BC                      4 S_L    then
//                   KAP (per-triangle kappa)         2 n_L^2
//   mixed solver:   FP64 X after the hierarchy (see solve_one_mixed)
// The FP64 solver preconditions with a V-cycle whose finest-level weights
// are the FP32-rounded edge weights: the preconditioner only has to be a
// fixed symmetric positive definite operator close to A, and the stencil
// apply and the residual of CG keep the FP64 weights, so the iterates still
// converge to the FP64 system's solution.  The V-cycle then reads half the
// weight bytes per pass.
enum { FX = 0, FR, FZ, FP, FQ, FWX, FWY, FP2, FWX32, FWY32 };  // fine arrays
__host__ __device__ inline int64_t pad_sz(int L) { return ((int64_t(1) << L) + 1) * ((int64_t(1) << L) + 1); }
__host__ __device__ inline int64_t half_sz(int L) { return (pad_sz(L) + 1) / 2; }  // FP32 grid in FP64 elements
__host__ __device__ inline int64_t coarse_sz(int L) { return 4 * pad_sz(L) + 2 * (int64_t(1) << (2 * L)); }
__host__ __device__ inline int64_t fine_sz(int l, bool split) { return 8 * pad_sz(l) + (split ? 2 * half_sz(l) : 0); }

__host__ __device__ inline int64_t coarse_off(int l, int L, bool split)
{
    int64_t o = fine_sz(l, split);
    for (int k = l - 1; k > L; --k) o += coarse_sz(k);
    return o;
}

// fine level and coarse hierarchy
__host__ __device__ inline int64_t hier_elems(int l, bool mixed)
{
    int64_t o = fine_sz(l, !mixed);
    for (int k = l - 1; k >= 1; --k) o += coarse_sz(k);
    return o;
}

// 9 x 9 inverse of the h = 1/4 operator, the FP64 V-cycle's coarsest solve
constexpr int64_t kCinvElems = 81;

__host__ __device__ inline int64_t slot_elems_hd(int l, bool mixed)
{
    // float slot: + FP64 X64 (2 floats per node) after an even offset;
    // double slot: + the coarse inverse, used when LDS has no room for it
    return hier_elems(l, mixed) + (mixed ? 2 * pad_sz(l) + 2 : kCinvElems);
}

int64_t solver_slot_elems(int l, bool mixed) { return slot_elems_hd(l, mixed); }

template <typename T, typename W = T>
struct Lv {
    W *wx, *wy;
    T *x, *b, *kap;
    int n, lg, s;
};

// Where a particle's arrays live.  Coarse levels L <= lds_top keep their
// four work arrays (WX WY XC BC) in LDS, finest of them first; after them
// come the first fine_n of the fine level's arrays in the order of how many
// passes of a PCG iteration touch them: the V-cycle's weights (read by five
// passes; the FP32 copies in the FP64 solver), Z and R (the V-cycle's
// unknown and right-hand side), the two search-direction buffers, Q, X, and
// last the FP64 weights of the FP64 solver (read by the stencil pass only).
// The per-triangle coefficients of coarse levels (setup only) and every
// other array stay in the global slot.
__host__ __device__ inline int fine_rank(int k, bool split)  // LDS priority of fine array k
{
    // X R Z P Q WX WY P2 WX32 WY32 -> split: 7 3 2 4 6 8 9 5 0 1; else 7 3 2 4 6 0 1 5
    const uint64_t t = split ? 0x1059864237ull : 0x51064237ull;
    return (int)((t >> (4 * k)) & 0xfu);
}
__host__ __device__ inline int fine_count(bool split) { return split ? 10 : 8; }
// elements before rank r in the LDS order
__host__ __device__ inline int64_t fine_prefix(int l, bool split, int r)
{
    if (!split) return r * pad_sz(l);
    return r <= 2 ? r * half_sz(l) : 2 * half_sz(l) + (r - 2) * pad_sz(l);
}
// offset of fine array k in the global slot
__host__ __device__ inline int64_t fine_slot_off(int l, int k)
{
    return k < FWX32 ? k * pad_sz(l) : 8 * pad_sz(l) + (k - FWX32) * half_sz(l);
}

template <typename T>
struct Map {
    T* slot;
    T* lds;
    int l;
    int lds_top;
    int fine_n;
    double* cinv;  // 9 x 9 inverse of the h = 1/4 operator (LDS or the slot), FP64 only
    T* ring;       // LDS rows of the fused row walks (null: the walks are off)
};

__host__ __device__ inline int64_t lds_coarse_elems(int top)
{
    int64_t o = 0;
    for (int k = 1; k <= top; ++k) o += 4 * pad_sz(k);
    return o;
}

// The residency for a budget of `budget` elements: the finest coarse level
// whose hierarchy fits, then as many fine arrays as fit in what is left.
// Never uses more than the budget, and applied to its own usage it returns
// the same residency (so a launch may pass the usage as the budget).
__host__ __device__ inline void lds_policy(int l, bool split, int64_t budget, int* top, int* fine_n)
{
    *fine_n = 0;
    *top = 0;
    if (budget <= 0) return;
    for (int t = l - 1; t >= 1; --t)
        if (lds_coarse_elems(t) <= budget) { *top = t; break; }
    const int64_t rem = budget - lds_coarse_elems(*top);
    int n = 0;
    while (n < fine_count(split) && fine_prefix(l, split, n + 1) <= rem) ++n;
    *fine_n = n;
}

__host__ __device__ inline int64_t lds_elems_used(int l, bool split, int64_t budget)
{
    int top, fine_n;
    lds_policy(l, split, budget, &top, &fine_n);
    return lds_coarse_elems(top) + fine_prefix(l, split, fine_n);
}

int64_t solver_lds_elems_used(int l, bool mixed, int64_t budget_elems)
{
    return lds_elems_used(l, !mixed, budget_elems);
}

template <typename T>
__device__ inline Map<T> make_map(T* slot, T* lds, int l, int64_t lds_budget_elems, double* cinv,
                                  T* ring = nullptr)
{
    Map<T> M;
    M.slot = slot;
    M.lds = lds;
    M.l = l;
    M.cinv = cinv;
    M.ring = ring;
    lds_policy(l, sizeof(T) == 8, lds ? lds_budget_elems : 0, &M.lds_top, &M.fine_n);
    return M;
}

template <typename T>
__device__ inline Lv<T> coarse_level(const Map<T>& M, int L)
{
    Lv<T> v;
    T* g = M.slot + coarse_off(M.l, L, sizeof(T) == 8);
    const int64_t S = pad_sz(L);
    T* base = (L <= M.lds_top) ? M.lds + (lds_coarse_elems(M.lds_top) - lds_coarse_elems(L)) : g;
    v.wx = base; v.wy = base + S; v.x = base + 2 * S; v.b = base + 3 * S;
    v.kap = g + 4 * S;
    v.n = 1 << L; v.lg = L; v.s = v.n + 1;
    return v;
}

// fine array k (FX .. FWY32) of the particle, in elements of T
template <typename T>
__device__ inline T* fine_array(const Map<T>& M, int k)
{
    const bool split = sizeof(T) == 8;
    const int r = fine_rank(k, split);
    return r < M.fine_n ? M.lds + lds_coarse_elems(M.lds_top) + fine_prefix(M.l, split, r)
                        : M.slot + fine_slot_off(M.l, k);
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

// the same on a level whose weights may be stored in a narrower type W
// (converted exactly to T before use)
template <typename T, typename W>
__device__ __forceinline__ T ldiag(const Lv<T, W>& L, int c)
{
    return T(L.wx[c - 1]) + T(L.wx[c]) + T(L.wy[c - L.s]) + T(L.wy[c]);
}

template <typename T, typename W>
__device__ __forceinline__ T lnb(const Lv<T, W>& L, const T* __restrict__ x, int c)
{
    return T(L.wx[c - 1]) * x[c - 1] + T(L.wx[c]) * x[c + 1] + T(L.wy[c - L.s]) * x[c - L.s]
         + T(L.wy[c]) * x[c + L.s];
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

// Synchronisation of the first wave alone: a wave's lanes see each other's
// LDS stores once the wave's own memory operations have completed, which
// the workgroup-scope fences wait for.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Working types whose V-cycle ends in an exact solve at h = 1/4
template <typename T>
constexpr bool kExactCoarse = sizeof(T) == 8;

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
                             int n, int lg, float* __restrict__ wx32 = nullptr, float* __restrict__ wy32 = nullptr)
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
        if (wx32) {  // FP32-rounded copies for the V-cycle of the FP64 solver
            wx32[t] = (float)vx;
            wy32[t] = (float)vy;
        }
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

// ------------------------------------------------------- column walk --
// On a level whose row width n divides the workgroup (BS = m n; used from
// h = 1/64 on) the CG
// stencil pass goes by columns: the m groups of n threads take m bands of
// rows, and thread i of a group owns column i of its band and walks it
// upward, keeping p and WY of the row below and of its own row in
// registers.  Each row of Z, P_old and WY is then loaded once per pass
// rather than three times (plus one row at each band's start).  Lane 0 of a
// group owns the boundary column and idles.  With m = 1 the row loop gives
// thread i the same nodes in the same order, and the walk evaluates the
// same expressions, so the results are bitwise the row loop's; with m > 1
// only the order of the inner product's terms differs.  (The Gauss-Seidel
// sweeps stay row loops: a column holds one node of a colour per two rows,
// so a walking sweep runs its division with half the lanes masked, which
// measured slower.)

// The walk indexes every array with one 32-bit offset, as the row loops do;
// left visible, the serial row index lets the compiler turn each access
// into a 64-bit pointer of its own, which costs registers the solver has
// not got.
__device__ __forceinline__ int opaque(int c)
{
    asm("" : "+v"(c));
    return c;
}

// p = z + beta p_old formed on the fly at the node and its neighbours,
// stored to Pn with q = A p; returns this thread's share of (p, q).  With X
// the pass also applies the pending x += xa p_old at its nodes.
template <int BS, bool NT, typename T>
__device__ double walk_apply(const Lv<T>& F, const T* __restrict__ Z, const T* __restrict__ Po, T beta,
                             T* __restrict__ Pn, T* __restrict__ Q, T* __restrict__ X = nullptr, T xa = T(0))
{
    const int n = F.n, s = F.s, m = BS / n;
    const int i = threadIdx.x & (n - 1), band = threadIdx.x / n;
    const int rows = (n - 2 + m) / m;  // ceil((n - 1) / m)
    const int j0 = 1 + band * rows, j1 = min(n, j0 + rows);
    double pq = 0.0;
    if (i == 0 || j0 >= j1) return pq;
    auto pn = [&](int q) { return fma(beta, Po[q], Z[q]); };
    const int c0 = (j0 - 1) * s + i;
    T pm = pn(c0), p0 = pn(c0 + s), wym = F.wy[c0];
#pragma unroll 1
    for (int j = j0; j < j1; ++j) {
        const int c = opaque(j * s + i);
        const T pp = pn(c + s), wyc = F.wy[c];
        const T v = (F.wx[c - 1] + F.wx[c] + wym + wyc) * p0
                  - (F.wx[c - 1] * pn(c - 1) + F.wx[c] * pn(c + 1) + wym * pm + wyc * pp);
        if constexpr (NT) {
            // on the walked levels p and q are read again only in later
            // passes: streaming stores keep them from pushing the rows the
            // walks reuse out of the L2 (on smaller levels they stay in the
            // caches until then, and plain stores are faster)
            __builtin_nontemporal_store(p0, &Pn[c]);
            __builtin_nontemporal_store(v, &Q[c]);
        } else {
            Pn[c] = p0;
            Q[c] = v;
        }
        if (X) X[c] += xa * Po[c];
        pq += (double)p0 * (double)v;
        pm = p0;
        p0 = pp;
        wym = wyc;
    }
    return pq;
}

// ------------------------------------------------------------ V-cycle --
template <int BS, typename T, typename W>
__device__ void smooth_colour(const Lv<T, W>& L, const T* __restrict__ b, T* __restrict__ x, int col,
                              bool first)
{
    // Each thread also stores its east neighbour (the other colour, value
    // unchanged), so the stores of a wave cover whole lines: a store of
    // every other double costs more than a full one.
    const int s = L.s;
    if (first) {  // the other colour is taken as zero
        MLS_FOR_COLOUR(L, col, {
            x[c] = b[c] / ldiag(L, c);
            x[c + 1] = T(0);
        })
    } else {
        MLS_FOR_COLOUR(L, col, {
            const T xe = x[c + 1];
            const T nb = T(L.wx[c - 1]) * x[c - 1] + T(L.wx[c]) * xe + T(L.wy[c - s]) * x[c - s]
                       + T(L.wy[c]) * x[c + s];
            x[c] = (b[c] + nb) / ldiag(L, c);
            x[c + 1] = xe;
        })
    }
}

// First black sweep after the coarse-grid correction x += P e.  A black
// node's four neighbours are red, and the corrected red values are read only
// by this sweep (the red sweep after it overwrites them), so the correction
// is interpolated at the neighbours on the fly and never stored.  At a red
// node (i', j') both indices are even (the coarse node itself) or both odd
// (the middle of a coarse diagonal edge, from (i'-1, j'-1) to (i'+1, j'+1)).
template <int BS, typename T, typename W>
__device__ void smooth_black_corrected(const Lv<T, W>& L, const Lv<T>& C, const T* __restrict__ b,
                                       T* __restrict__ x)
{
    const int s = L.s, sc = C.s;
    const T* __restrict__ e = C.x;
    auto pe = [&](int ii, int jj) -> T {
        const int q = (jj >> 1) * sc + (ii >> 1);
        return (ii & 1) ? T(0.5) * (e[q] + e[q + sc + 1]) : e[q];
    };
    MLS_FOR_COLOUR(L, 1, {
        const T xe = x[c + 1];
        const T nb = T(L.wx[c - 1]) * (x[c - 1] + pe(i - 1, j)) + T(L.wx[c]) * (xe + pe(i + 1, j))
                   + T(L.wy[c - s]) * (x[c - s] + pe(i, j - 1)) + T(L.wy[c]) * (x[c + s] + pe(i, j + 1));
        x[c] = (b[c] + nb) / ldiag(L, c);
        x[c + 1] = xe;  // whole-line stores, as in smooth_colour (the red values are dead here)
    })
}

// Down-leg on level L: (red, black)^nu, then the restriction of the residual
// into the coarser level's right-hand side C.b.  pre_red_done: the caller
// has already done the first red sweep (fused with its vector updates).
template <int BS, typename T, typename W>
__device__ void down_step(const Lv<T, W>& L, const Lv<T>& C, const T* __restrict__ b, T* __restrict__ x,
                          int nu, bool pre_red_done)
{
    for (int sw = 0; sw < nu; ++sw) {
        if (!(sw == 0 && pre_red_done)) {
            smooth_colour<BS>(L, b, x, 0, sw == 0);
            __syncthreads();
        }
        smooth_colour<BS>(L, b, x, 1, false);
        __syncthreads();
    }
    // restriction of the residual (P^T of P1 interpolation), formed in the
    // same pass.  The last sweep was black, and a Gauss-Seidel sweep
    // satisfies the equations of the nodes it updates, so the black
    // residuals vanish: of the seven fine nodes P^T gathers only the three
    // red ones carry a residual, the coarse node itself and its two
    // neighbours along the triangle diagonal.
    const int s = L.s;
    auto res = [&](int q) { return b[q] - (ldiag(L, q) * x[q] - lnb(L, x, q)); };
    MLS_FOR_INTERIOR(C, {
        const int f = (2 * j) * s + 2 * i;
        C.b[c] = res(f) + T(0.5) * (res(f + s + 1) + res(f - s - 1));
    })
    __syncthreads();
}

// Up-leg on level L after the coarser level C was solved: (black, red)^nu
// with the coarse correction folded into the first black sweep.  With
// want_dot the last red sweep also returns (b, x) over all interior nodes
// (black values are final there, so the pass can read them).
template <int BS, typename T, typename W>
__device__ double up_step(const Lv<T, W>& L, const Lv<T>& C, const T* __restrict__ b, T* __restrict__ x,
                          int nu, bool want_dot, double* red)
{
    double dot = 0.0;
    for (int sw = 0; sw < nu; ++sw) {
        if (sw == 0) smooth_black_corrected<BS>(L, C, b, x);
        else smooth_colour<BS>(L, b, x, 1, false);
        __syncthreads();
        if (sw == nu - 1 && want_dot) {
            double d = 0.0;
            MLS_FOR_INTERIOR(L, {
                T z;
                if (((i + j) & 1) == 0) {
                    z = (b[c] + lnb(L, x, c)) / ldiag(L, c);
                } else {
                    z = x[c];
                }
                x[c] = z;  // black nodes store their own value: whole-line stores
                d += (double)b[c] * (double)z;
            })
            dot = block_sum<BS>(d, red);  // includes the barrier
        } else {
            smooth_colour<BS>(L, b, x, 0, false);
            __syncthreads();
        }
    }
    return dot;
}

// ------------------------------------------------------- fused row walks --
// On a large level (n >= 256) the down-leg (optional residual update r -= a q,
// red sweep from a zero start, black sweep, restriction of the residual)
// and the up-leg (black sweep with the coarse correction, red sweep, the
// dot (b, z)) each run as one pass over the rows instead of three and two.
// Thread t of a band owns the column pair (2t, 2t+1) of every row of the
// band, so each row step gives every thread one red and one black node.
// Going up row j, the down walk updates the residual of row j and its red
// node, the black node of row j-1 (its red neighbours are final), the red
// residual of row j-2 (its black neighbours are final) and, one step later
// (the residuals of a row come from neighbouring threads), the coarse
// right-hand side of coarse row (j-4)/2.  A node's own column lives in the
// thread's registers, the neighbouring threads' values pass through a ring
// of LDS rows, with one barrier per row step.  Every node evaluates the
// same expression as the separate sweeps, so the iterates are bitwise
// theirs; only the order of the terms of (b, z) differs.
//
// The m = BS / (n/2) bands walk their row ranges [j0, j1) in lock step.  A
// band first recomputes, without storing, the three rows below j0 from the
// residual update's inputs, which the band below overwrites only at the end
// of its walk; above j1 it recomputes the red and black values from the
// updated residual, which the band above stored in its first steps.  The up
// walk reads only values that no band writes during it (the down walk's z,
// the right-hand side, the coarse correction) and writes the new z to a
// second array, so its bands need no ordering at all.
template <int BS>
__device__ __forceinline__ bool walk_level(int n, int nu)
{
    return nu == 1 && n >= 256 && BS % (n >> 1) == 0;
}

// LDS elements of the walks on a level of width n: per band four rows of
// the node values and four rows of the red residuals (one per thread)
__host__ __device__ inline int64_t walk_ring_elems_level(int bs, int n)
{
    const int64_t m = bs / (n >> 1);
    return m * (4 * (int64_t)(n + 1) + 4 * (int64_t)((n >> 1) + 1));
}
// the most any walked level of a hierarchy with finest level l needs
__host__ __device__ inline int64_t walk_ring_elems(int bs, int l)
{
    int64_t e = 0;
    for (int L = l; L >= 8; --L) {
        const int n = 1 << L;
        if (bs % (n >> 1) == 0) {
            const int64_t v = walk_ring_elems_level(bs, n);
            if (v > e) e = v;
        }
    }
    return e;
}

// One band's rows: [j0, j1), the ring offset of the band, this thread's
// pair.  A band has n / m rows, an even number, so every band starts on an
// odd row and the walks can unroll two row steps of fixed parity.
struct WalkRows {
    int t, j0, j1;
    int64_t ring_off;
};
template <int BS>
__device__ __forceinline__ WalkRows walk_rows(int n)
{
    const int P = n >> 1, m = BS / P;
    const int band = threadIdx.x / P;
    WalkRows w;
    w.t = threadIdx.x - band * P;
    const int rows = n / m;
    w.j0 = 1 + band * rows;
    w.j1 = min(n, w.j0 + rows);
    w.ring_off = (int64_t)band * (4 * (n + 1) + 4 * (P + 1));
    return w;
}

template <int K>
using Par = std::integral_constant<int, K>;

// The walked levels never sit in LDS (a row of 257 values already exceeds
// the residency budgets), so the walks address their arrays as global
// memory and their rows as LDS: global and LDS instructions instead of flat
// ones, which also lets the compiler keep them apart.
template <typename T>
using gmem = T __attribute__((address_space(1)))*;
template <typename T>
using lmem = T __attribute__((address_space(3)))*;

// The barrier between row steps: it orders the LDS ring only, so the
// global loads and stores of a step stay in flight across it (a full
// barrier would wait for every store to be acknowledged).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Down-leg of a V(1,1) cycle on level L into the coarser level's right-hand
// side C.b.  With Q: b -= alpha Q first (the CG residual update; b is
// updated in place) and, with X and Pn, also X += alpha Pn (the mixed
// solver's iterate).  Without Q, b is only read.  x receives z.  In a step
// on row j every phase works on the thread's column of parity j: the red
// node of row j, the black node of row j-1 and the red node of row j-2 all
// sit in it.  The node values of the last four rows are kept in the LDS
// ring (the thread's own ones too); the weights come from registers on the
// finest level and from memory on a walked coarse level (see below).
template <int BS, bool FINE, typename T, typename W>
__device__ void walk_down(const Lv<T, W>& L, const Lv<T>& C, T* __restrict__ b, const T* __restrict__ Q, T alpha,
                          T* __restrict__ x, T* __restrict__ X, const T* __restrict__ Pn, T* __restrict__ ring)
{
    const int n = L.n, s = L.s, P = n >> 1, sc = C.s, nc = C.n;
    const WalkRows w = walk_rows<BS>(n);
    const int t = w.t, j0 = w.j0, j1 = w.j1, ca = 2 * t;
    const lmem<T> lring = (lmem<T>)ring;
    const lmem<T> zr = lring + w.ring_off;  // node values, 4 rows of s
    const lmem<T> rr = zr + 4 * s;          // red residuals, 4 rows of P + 1
    // columns 0 and n of the rows are never written: they read as the zero boundary
    for (int k = threadIdx.x; k < walk_ring_elems_level(BS, n); k += BS) lring[k] = T(0);
    __syncthreads();
    const gmem<const W> wx = (gmem<const W>)L.wx;
    const gmem<const W> wy = (gmem<const W>)L.wy;
    const gmem<T> gb = (gmem<T>)b;
    const gmem<const T> gQ = (gmem<const T>)Q;
    const gmem<T> gx = (gmem<T>)x;
    const gmem<T> gX = (gmem<T>)X;
    const gmem<const T> gPn = (gmem<const T>)Pn;
    const gmem<T> gCb = (gmem<T>)C.b;
    T r0[2] = {T(0), T(0)}, r1[2] = {T(0), T(0)}, r2[2] = {T(0), T(0)};  // updated residual, rows j .. j-2
    // On the finest level (FINE; FP32 weights in both solvers) the weights
    // of the thread's columns are read from global memory once per row and
    // carried through the three steps that use them: wx of columns
    // ca-1 .. ca+1 for rows j .. j-2, wy of columns ca, ca+1 for rows
    // j .. j-3.  Read again from memory, those rows fall out of the L2 when
    // every CU of an XCD walks its own particle.  On the walked coarse level
    // (FP64 weights in the FP64 solver) the registers are dearer than the
    // re-reads, and the weights are read where they are used.
    constexpr bool win = FINE;
    W x0[3], x1[3], x2[3], y0[2], y1[2], y2[2], y3[2];
    // wx of row j - r, column ca - 1 + u; wy of row j - r, column ca + u
    auto WX = [&](int j, int r, int u) -> T {
        if constexpr (win) return T(r == 0 ? x0[u] : r == 1 ? x1[u] : x2[u]);
        else return T(wx[(j - r) * s + ca - 1 + u]);
    };
    auto WY = [&](int j, int r, int u) -> T {
        if constexpr (win) return T(r == 0 ? y0[u] : r == 1 ? y1[u] : r == 2 ? y2[u] : y3[u]);
        else return T(wy[(j - r) * s + ca + u]);
    };
    auto load_w = [&](int jj, W* xr, W* yr) {
        const bool in = jj >= 0 && jj <= n - 1;
        const int c = jj * s + ca;
        xr[0] = in && ca > 0 ? wx[c - 1] : W(0);
        xr[1] = in ? wx[c] : W(0);
        xr[2] = in ? wx[c + 1] : W(0);
        yr[0] = in ? wy[c] : W(0);
        yr[1] = in ? wy[c + 1] : W(0);
    };
    if constexpr (win) {
        load_w(j0 - 4, x0, y0);
#pragma unroll
        for (int u = 0; u < 3; ++u) x1[u] = x2[u] = W(0);
        y1[0] = y1[1] = y2[0] = y2[1] = y3[0] = y3[1] = W(0);
    }
    auto body = [&](auto par, int j) {
        constexpr int k = decltype(par)::value;  // the active column: ca + k
        r2[0] = r1[0]; r2[1] = r1[1]; r1[0] = r0[0]; r1[1] = r0[1]; r0[0] = T(0); r0[1] = T(0);
        if constexpr (win) {
#pragma unroll
            for (int u = 0; u < 3; ++u) { x2[u] = x1[u]; x1[u] = x0[u]; }
            y3[0] = y2[0]; y3[1] = y2[1]; y2[0] = y1[0]; y2[1] = y1[1]; y1[0] = y0[0]; y1[1] = y0[1];
            load_w(j, x0, y0);
        }
        const bool active = ca + k > 0;  // column 0 is the boundary
        auto Z = [&](int jj, int i) -> T __attribute__((address_space(3)))& { return zr[(jj & 3) * s + i]; };
        if (j == n) {  // the top boundary row, read by the black sweep and the residuals below it
            Z(n, ca) = T(0);
            Z(n, ca + 1) = T(0);
        }
        // ---- row j: residual update and the red node
        if (j >= 1 && j <= n - 1 && j <= j1 + 2) {
            const int c = j * s + ca;
            if (Q && j < j1) {
                r0[0] = gb[c] - alpha * gQ[c];
                r0[1] = gb[c + 1] - alpha * gQ[c + 1];
                if (j >= j0) {
                    if (ca > 0) gb[c] = r0[0];
                    gb[c + 1] = r0[1];
                    if (X) {
                        gX[c] += alpha * gPn[c];
                        gX[c + 1] += alpha * gPn[c + 1];
                    }
                }
            } else {  // no update, or rows above the band (updated there already)
                r0[0] = gb[c];
                r0[1] = gb[c + 1];
            }
            if (active)
                Z(j, ca + k) = r0[k] / (WX(j, 0, k) + WX(j, 0, k + 1) + WY(j, 1, k) + WY(j, 0, k));
        }
        // ---- row j-1: the black node (red neighbours final)
        const int jb = j - 1;
        if (jb >= 1 && jb <= n - 1 && jb >= j0 - 2 && jb <= j1 + 1) {
            const int i = ca + k;
            if (active) {
                const T nb = WX(j, 1, k) * Z(jb, i - 1) + WX(j, 1, k + 1) * Z(jb, i + 1) + WY(j, 2, k) * Z(jb - 1, i)
                           + WY(j, 1, k) * Z(j, i);
                Z(jb, i) = (r1[k] + nb) / (WX(j, 1, k) + WX(j, 1, k + 1) + WY(j, 2, k) + WY(j, 1, k));
            }
            if (jb >= j0 && jb < j1) {  // row j-1 is final: store both columns (streaming)
                if (ca > 0) __builtin_nontemporal_store((T)Z(jb, ca), &gx[jb * s + ca]);
                __builtin_nontemporal_store((T)Z(jb, ca + 1), &gx[jb * s + ca + 1]);
            }
        }
        // ---- row j-2: the red residual (black neighbours final)
        const int jc = j - 2;
        if (jc >= 1 && jc <= n - 1 && jc >= j0 - 1 && jc <= j1 && active) {
            const int i = ca + k;
            const T d = WX(j, 2, k) + WX(j, 2, k + 1) + WY(j, 3, k) + WY(j, 2, k);
            const T lnb = WX(j, 2, k) * Z(jc, i - 1) + WX(j, 2, k + 1) * Z(jc, i + 1) + WY(j, 3, k) * Z(jc - 1, i)
                        + WY(j, 2, k) * Z(jc + 1, i);
            rr[(jc & 3) * (P + 1) + t] = r2[k] - (d * Z(jc, i) - lnb);
        }
        // ---- coarse row (j-4)/2: restriction of the red residuals
        if (k == 0) {
            const int J = (j - 4) >> 1;
            if (J >= 1 && J <= nc - 1 && 2 * J >= j0 && 2 * J < j1 && t >= 1 && t <= nc - 1) {
                const T a0 = rr[((2 * J) & 3) * (P + 1) + t];
                const T ap = rr[((2 * J + 1) & 3) * (P + 1) + t];
                const T am = rr[((2 * J - 1) & 3) * (P + 1) + t - 1];
                gCb[J * sc + t] = a0 + T(0.5) * (ap + am);
            }
        }
        // the band above stored its first three rows (the rows this band's
        // walk ends on) in steps 3 to 5: one full barrier after them makes
        // those stores visible; every other step orders the LDS ring only
        if (j - (j0 - 3) == 6) __syncthreads();
        else lds_barrier();
    };
    // rows j0 - 3 (even) .. j1 + 3
#pragma unroll 1
    for (int j = j0 - 3; j <= j0 + (n / (BS / P)) + 4; j += 2) {
        body(Par<0>{}, j);
        body(Par<1>{}, j + 1);
    }
    __syncthreads();  // z, the updated residual and C.b are complete
}

// Up-leg of a V(1,1) cycle on level L after the coarser level was solved
// (its correction e, row stride sc): the black sweep with the correction
// interpolated at the red neighbours, then the red sweep, reading the down
// walk's z from xo and writing the new z to xn.  Returns (b, z) over the
// interior nodes when want_dot.  In a step on row j both phases work on the
// thread's column of parity j + 1: the black node of row j and the red node
// of row j - 1.  New values pass through the LDS ring as in walk_down.
template <int BS, bool FINE, typename T, typename W>
__device__ double walk_up(const Lv<T, W>& L, const T* __restrict__ e, int sc, const T* __restrict__ b,
                          const T* __restrict__ xo, T* __restrict__ xn, bool want_dot, T* __restrict__ ring,
                          double* red)
{
    const int n = L.n, s = L.s;
    const WalkRows w = walk_rows<BS>(n);
    const int j0 = w.j0, j1 = w.j1, ca = 2 * w.t;
    const lmem<T> lring = (lmem<T>)ring;
    const lmem<T> zb = lring + w.ring_off;  // new values, 4 rows of s
    for (int k = threadIdx.x; k < walk_ring_elems_level(BS, n); k += BS) lring[k] = T(0);
    __syncthreads();
    const gmem<const W> wx = (gmem<const W>)L.wx;
    const gmem<const W> wy = (gmem<const W>)L.wy;
    const gmem<const T> ge = (gmem<const T>)e;
    const gmem<const T> gbv = (gmem<const T>)b;
    const gmem<const T> xo_ = (gmem<const T>)xo;
    const gmem<T> xn_ = (gmem<T>)xn;
    auto pe = [&](int ii, int jj) -> T {
        const int q = (jj >> 1) * sc + (ii >> 1);
        return (ii & 1) ? T(0.5) * (ge[q] + ge[q + sc + 1]) : ge[q];
    };
    T b0[2] = {T(0), T(0)}, b1[2] = {T(0), T(0)};  // right-hand side of rows j, j-1
    double dot = 0.0;
    // As in walk_down, on the finest level each row's weights of the
    // thread's columns (wx of columns ca-1 .. ca+1 for rows j, j-1; wy of
    // columns ca, ca+1 for rows j .. j-2) are read from global memory once
    // and carried in registers; in the FP64 solver so is the down walk's z
    // of the thread's own two columns (rows j-1 .. j+1), which in the mixed
    // solver would cost the kernel an occupancy step.
    constexpr bool win = FINE;
    constexpr bool zwin = FINE && sizeof(W) < sizeof(T);
    W x0[3], x1[3], y0[2], y1[2], y2[2];
    T zm[2], zc[2], zp[2];  // xo of columns ca, ca+1: rows j-1, j, j+1
    auto WX = [&](int j, int r, int u) -> T {  // wx of row j - r, column ca - 1 + u
        if constexpr (win) return T(r == 0 ? x0[u] : x1[u]);
        else return T(wx[(j - r) * s + ca - 1 + u]);
    };
    auto WY = [&](int j, int r, int u) -> T {  // wy of row j - r, column ca + u
        if constexpr (win) return T(r == 0 ? y0[u] : r == 1 ? y1[u] : y2[u]);
        else return T(wy[(j - r) * s + ca + u]);
    };
    auto XO = [&](int j, int r, int u) -> T {  // xo of row j + r (r = -1, 0, 1), column ca + u
        if constexpr (zwin) return r < 0 ? zm[u] : r == 0 ? zc[u] : zp[u];
        else return xo_[(j + r) * s + ca + u];
    };
    auto load_w = [&](int jj, W* xr, W* yr) {
        const bool in = jj >= 0 && jj <= n - 1;
        const int c = jj * s + ca;
        xr[0] = in && ca > 0 ? wx[c - 1] : W(0);
        xr[1] = in ? wx[c] : W(0);
        xr[2] = in ? wx[c + 1] : W(0);
        yr[0] = in ? wy[c] : W(0);
        yr[1] = in ? wy[c + 1] : W(0);
    };
    auto load_z = [&](int jj, T* zr_) {
        const bool in = jj >= 0 && jj <= n;
        zr_[0] = in ? xo_[jj * s + ca] : T(0);
        zr_[1] = in ? xo_[jj * s + ca + 1] : T(0);
    };
    if constexpr (win) {
        load_w(j0 - 2, x0, y0);
        y1[0] = y1[1] = W(0);
        if constexpr (zwin) {
            load_z(j0 - 2, zc);
            load_z(j0 - 1, zp);
        }
    }
    auto body = [&](auto par, int j) {
        constexpr int k = 1 - decltype(par)::value;  // the active column: ca + k
        b1[0] = b0[0]; b1[1] = b0[1]; b0[0] = T(0); b0[1] = T(0);
        if constexpr (win) {
#pragma unroll
            for (int u = 0; u < 3; ++u) x1[u] = x0[u];
            y2[0] = y1[0]; y2[1] = y1[1]; y1[0] = y0[0]; y1[1] = y0[1];
            load_w(j, x0, y0);
            if constexpr (zwin) {
                zm[0] = zc[0]; zm[1] = zc[1]; zc[0] = zp[0]; zc[1] = zp[1];
                load_z(j + 1, zp);
            }
        }
        auto Z = [&](int jj, int i) -> T __attribute__((address_space(3)))& { return zb[(jj & 3) * s + i]; };
        const int i = ca + k;
        if (j == n) {  // the top boundary row, read by the red sweep below it
            Z(n, ca) = T(0);
            Z(n, ca + 1) = T(0);
        }
        // ---- row j: the black node, corrected
        if (j >= 1 && j <= n - 1 && j <= j1) {
            const int c0 = j * s + ca;
            b0[0] = gbv[c0];
            b0[1] = gbv[c0 + 1];
            if (i > 0) {
                const int c = c0 + k;
                // the horizontal neighbour outside the pair is the
                // neighbouring thread's: read from memory (this row, cached)
                const T xw = k == 0 ? xo_[c - 1] : XO(j, 0, 0);
                const T xe = k == 0 ? XO(j, 0, 1) : xo_[c + 1];
                const T nb = WX(j, 0, k) * (xw + pe(i - 1, j)) + WX(j, 0, k + 1) * (xe + pe(i + 1, j))
                           + WY(j, 1, k) * (XO(j, -1, k) + pe(i, j - 1)) + WY(j, 0, k) * (XO(j, 1, k) + pe(i, j + 1));
                Z(j, i) = (b0[k] + nb) / (WX(j, 0, k) + WX(j, 0, k + 1) + WY(j, 1, k) + WY(j, 0, k));
            }
        }
        // ---- row j-1: the red node (black neighbours new); the row is then final
        const int jr = j - 1;
        if (jr >= j0 && jr < j1) {
            if (i > 0) {
                const T lnb = WX(j, 1, k) * Z(jr, i - 1) + WX(j, 1, k + 1) * Z(jr, i + 1) + WY(j, 2, k) * Z(jr - 1, i)
                            + WY(j, 1, k) * Z(j, i);
                Z(jr, i) = (b1[k] + lnb) / (WX(j, 1, k) + WX(j, 1, k + 1) + WY(j, 2, k) + WY(j, 1, k));
            }
            const T za = Z(jr, ca), zbb = Z(jr, ca + 1);
            if (ca > 0) __builtin_nontemporal_store(za, &xn_[jr * s + ca]);
            __builtin_nontemporal_store(zbb, &xn_[jr * s + ca + 1]);
            // column 0 is the boundary: its right-hand side entry is never
            // written and may hold a stale word of another level's layout
            // (any bit pattern, NaN included), so it stays out of the dot
            if (want_dot) dot += (ca > 0 ? (double)b1[0] * (double)za : 0.0) + (double)b1[1] * (double)zbb;
        }
        lds_barrier();  // the walk reads no global value another thread writes
    };
    // rows j0 - 1 (even) .. j1
#pragma unroll 1
    for (int j = j0 - 1; j <= j0 + (n / (BS / (n >> 1))); j += 2) {
        body(Par<0>{}, j);
        body(Par<1>{}, j + 1);
    }
    __syncthreads();  // the new z is complete
    return want_dot ? block_sum<BS>(dot, red) : 0.0;
}

// The V-cycle's coarsest level is h = 1/4 (nine unknowns), solved exactly
// with the inverse of its operator, formed once per particle in FP64 by the
// first wave: Gauss-Jordan sweeps in place over the 9 x 9 array (the
// operator is a symmetric M-matrix, so no pivoting is needed).  Unknown
// u = 3 (j - 1) + (i - 1).
template <int BS, typename T, typename W>
__device__ void build_coarse_inverse(const Lv<T, W>& L, double* cinv)
{
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x, s = L.s;
        for (int e = lane; e < 81; e += 64) {
            const int u = e / 9, v = e % 9;
            const int i = u % 3 + 1, j = u / 3 + 1, c = j * s + i;
            double a = 0.0;
            if (v == u) a = (double)ldiag(L, c);
            else if (v == u - 1 && i > 1) a = -(double)L.wx[c - 1];
            else if (v == u + 1 && i < 3) a = -(double)L.wx[c];
            else if (v == u - 3) a = -(double)L.wy[c - s];
            else if (v == u + 3) a = -(double)L.wy[c];
            cinv[e] = a;
        }
        wave_sync();
        // new value of entry e under the sweep on pivot p (r = 1 / pivot)
        auto swept = [&](int e, int p, double r) {
            const int u = e / 9, v = e % 9;
            if (u == p && v == p) return r;
            if (u == p) return cinv[9 * p + v] * r;
            if (v == p) return -cinv[9 * u + p] * r;
            return cinv[e] - cinv[9 * u + p] * cinv[9 * p + v] * r;
        };
        const int e1 = lane + 64;  // lanes 0..16 own a second entry
        for (int p = 0; p < 9; ++p) {
            const double r = 1.0 / cinv[9 * p + p];
            const double n0 = swept(lane, p, r);
            const double n1 = e1 < 81 ? swept(e1, p, r) : 0.0;
            wave_sync();
            cinv[lane] = n0;
            if (e1 < 81) cinv[e1] = n1;
            wave_sync();
        }
    }
    __syncthreads();
}

// x = A^{-1} b on the h = 1/4 level L (nine threads)
template <int BS, typename T, typename W>
__device__ void coarse_exact(const Lv<T, W>& L, const T* __restrict__ b, T* __restrict__ x, const double* cinv)
{
    if (threadIdx.x < 9) {
        const int s = L.s, u = threadIdx.x;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) v += cinv[9 * u + q] * (double)b[(q / 3 + 1) * s + q % 3 + 1];
        x[(u / 3 + 1) * s + u % 3 + 1] = T(v);
    }
    __syncthreads();
}

// One V-cycle z = V r on the hierarchy of M whose finest level is F (its
// weights of type W).  See down_step and up_step for pre_red_done and
// want_dot.
template <int BS, typename T, typename W>
__device__ double vcycle(const Map<T>& M, const Lv<T, W>& F, const T* __restrict__ rhs, T* __restrict__ sol,
                         int nu, bool pre_red_done, bool want_dot, double* red)
{
    const int l = M.l;
    if (l == 1) {  // the fine level is the coarsest: one unknown, exact
        if (threadIdx.x == 0) {
            const int c = F.s + 1;
            sol[c] = T((double)rhs[c] / (double)ldiag(F, c));
        }
        __syncthreads();
        double d = 0.0;
        if (want_dot) {
            MLS_FOR_INTERIOR(F, { d += (double)rhs[c] * (double)sol[c]; })
            d = block_sum<BS>(d, red);
        }
        return d;
    }
    if (kExactCoarse<T> && l == 2) {  // the fine level is the coarsest: exact
        coarse_exact<BS>(F, rhs, sol, M.cinv);
        double d = 0.0;
        if (want_dot) {
            MLS_FOR_INTERIOR(F, { d += (double)rhs[c] * (double)sol[c]; })
            d = block_sum<BS>(d, red);
        }
        return d;
    }
    // FP64 hierarchies stop at h = 1/4 and solve it exactly; FP32 ones go
    // down to the single unknown of h = 1/2 (fewer registers in that kernel)
    constexpr int Lc = kExactCoarse<T> ? 2 : 1;
    down_step<BS>(F, coarse_level(M, l - 1), rhs, sol, nu, pre_red_done);
    for (int Lk = l - 1; Lk > Lc; --Lk) {
        const Lv<T> L = coarse_level(M, Lk);
        down_step<BS>(L, coarse_level(M, Lk - 1), L.b, L.x, nu, false);
    }
    {
        const Lv<T> C = coarse_level(M, Lc);
        if constexpr (kExactCoarse<T>) {
            coarse_exact<BS>(C, C.b, C.x, M.cinv);
        } else {  // one unknown at (1,1), solved in FP64
            if (threadIdx.x == 0) {
                const int c = C.s + 1;
                C.x[c] = T((double)C.b[c] / (double)diag_at(C.wx, C.wy, c, C.s));
            }
            __syncthreads();
        }
    }
    for (int Lk = Lc + 1; Lk <= l - 1; ++Lk) {
        const Lv<T> L = coarse_level(M, Lk);
        up_step<BS>(L, coarse_level(M, Lk - 1), L.b, L.x, nu, false, red);
    }
    return up_step<BS>(F, coarse_level(M, l - 1), rhs, sol, nu, want_dot, red);
}

// The V(1,1) cycle with the fused row walks on every level that has them
// (walk_down / walk_up); the smaller levels keep the separate sweeps.  The
// finest level's up-leg writes z into zn, which the caller then takes as its
// z; a walked coarse level keeps its up-leg's result in its coarsening
// buffer (free after the set-up).  With Q the finest down walk first
// updates rhs -= alpha Q (and X += alpha Pn).  Returns (rhs, z) when
// want_dot.
template <int BS, typename T, typename W>
__device__ double vcycle_walk(const Map<T>& M, const Lv<T, W>& F, T* rhs, const T* Q, T alpha, T* X, const T* Pn,
                              T* sol, T* zn, bool want_dot, double* red)
{
    const int l = M.l;
    constexpr int Lc = kExactCoarse<T> ? 2 : 1;
    auto walked = [&](int L) { return walk_level<BS>(1 << L, 1); };
    auto result = [&](int L) {  // level L's z after its up-leg
        Lv<T> V = coarse_level(M, L);
        if (walked(L)) V.x = V.kap;
        return V;
    };
    walk_down<BS, true>(F, coarse_level(M, l - 1), rhs, Q, alpha, sol, X, Pn, M.ring);
    for (int Lk = l - 1; Lk > Lc; --Lk) {
        const Lv<T> L = coarse_level(M, Lk);
        if (walked(Lk))
            walk_down<BS, false>(L, coarse_level(M, Lk - 1), L.b, (const T*)nullptr, T(0), L.x, (T*)nullptr,
                          (const T*)nullptr, M.ring);
        else
            down_step<BS>(L, coarse_level(M, Lk - 1), L.b, L.x, 1, false);
    }
    {
        const Lv<T> C = coarse_level(M, Lc);
        if constexpr (kExactCoarse<T>) {
            coarse_exact<BS>(C, C.b, C.x, M.cinv);
        } else {  // one unknown at (1,1), solved in FP64
            if (threadIdx.x == 0) {
                const int c = C.s + 1;
                C.x[c] = T((double)C.b[c] / (double)diag_at(C.wx, C.wy, c, C.s));
            }
            __syncthreads();
        }
    }
    for (int Lk = Lc + 1; Lk <= l - 1; ++Lk) {
        const Lv<T> L = coarse_level(M, Lk);
        const Lv<T> Cc = result(Lk - 1);
        if (walked(Lk)) walk_up<BS, false>(L, Cc.x, Cc.s, L.b, L.x, L.kap, false, M.ring, red);
        else up_step<BS>(L, Cc, L.b, L.x, 1, false, red);
    }
    const Lv<T> Cf = result(l - 1);
    return walk_up<BS, true>(F, Cf.x, Cf.s, rhs, sol, zn, want_dot, M.ring, red);
}

// ------------------------------------------------------- setup & obs --
template <int BS, typename T, typename KT>
__device__ void setup_hierarchy(const Map<T>& M, const Lv<T>& F, const KT* __restrict__ kap,
                                float* wx32 = nullptr, float* wy32 = nullptr, bool walks = false)
{
    const int l = M.l;
    edge_weights<BS>(kap, F.wx, F.wy, F.n, F.lg, wx32, wy32);
    if (l >= 2) {
        Lv<T> C = coarse_level(M, l - 1);
        coarsen_kappa<BS>(kap, C.kap, l - 1);
        __syncthreads();
        for (int L = l - 1; L >= 1; --L) {
            Lv<T> V = coarse_level(M, L);
            edge_weights<BS>(V.kap, V.wx, V.wy, V.n, V.lg);
            zero_boundary<BS>(V.x, V.n);
            if (L >= 2) coarsen_kappa<BS>(V.kap, coarse_level(M, L - 1).kap, L - 1);
            __syncthreads();
        }
        // a walked level's coefficients are dead now: the buffer takes the
        // up-leg's z, whose boundary must read zero
        if (walks)
            for (int L = l - 1; L >= 8; --L)
                if (walk_level<BS>(1 << L, 1)) zero_boundary<BS>(coarse_level(M, L).kap, 1 << L);
        __syncthreads();
    }
}

// One particle's solve: its level, coefficient row and output rows.
struct Job {
    int l;
    const void* kap;     // n_e coefficients (double, or float for mixed)
    double* G;           // N_obs
    double* p_out;       // M or null
    int8_t* status;      // 1 or null
    int32_t* iters;      // 1 or null
    const double* y;     // data for the fused potential, or null
    double* phi;         // 1 or null
    const int32_t* obs_idx;
    const double* obs_w;
};

struct Common {
    int nobs;
    double inv_sigma;
    double tol2;
    int max_iters;
    int nu;
};

// J.G[o] += alpha (observation o of p): the observations of the iterate
// gathered step by step (thread o owns observation o, as in
// observe_and_store)
template <int BS>
__device__ void observe_step(const Job& J, const Common& C, const double* P, double alpha)
{
    for (int o = threadIdx.x; o < C.nobs; o += BS) {
        double g = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) g += J.obs_w[3 * o + k] * P[J.obs_idx[3 * o + k]];
        J.G[o] += alpha * g;
    }
}

// Observations, potential, status.  FROM_X: the observations are taken
// from the solution X; otherwise J.G already holds them (observe_step) and
// X is not read.
template <int BS, bool FROM_X = true, typename T>
__device__ void observe_and_store(const Job& J, const Common& C, const T* X, int n, int8_t st, int it,
                                  double* red)
{
    double ph = 0.0;
    for (int o = threadIdx.x; o < C.nobs; o += BS) {
        double g = 0.0;
        if constexpr (FROM_X) {
#pragma unroll
            for (int k = 0; k < 3; ++k) g += J.obs_w[3 * o + k] * (double)X[J.obs_idx[3 * o + k]];
            J.G[o] = g;
        } else {
            g = J.G[o];
        }
        if (J.y) {
            const double r = (J.y[o] - g) * C.inv_sigma;
            ph += r * r;
        }
    }
    if (FROM_X && J.p_out) {
        const int64_t M = (int64_t)(n - 1) * (n - 1);
        for (int64_t t = threadIdx.x; t < M; t += BS) {
            const int j = 1 + (int)(t / (n - 1)), i = 1 + (int)(t % (n - 1));
            J.p_out[t] = (double)X[j * (n + 1) + i];
        }
    }
    if (J.y) ph = block_sum<BS>(ph, red);
    if (threadIdx.x == 0) {
        if (J.status) *J.status = st;
        if (J.iters) *J.iters = it;
        if (J.phi) *J.phi = 0.5 * ph;
    }
    __syncthreads();
}

template <typename T>
__device__ inline Lv<T> fine_level(const Map<T>& M)
{
    Lv<T> F;
    F.wx = fine_array(M, FWX); F.wy = fine_array(M, FWY);
    F.x = fine_array(M, FZ); F.b = fine_array(M, FR); F.kap = nullptr;
    F.n = 1 << M.l; F.lg = M.l; F.s = F.n + 1;
    return F;
}

// ---------------------------------------------------------- FP64 solve --
template <int BS, int WK, bool KEEP_X>
__device__ void solve_one_f64(const Map<double>& M, const Job& J, const Common& C, double* red)
{
    const int l = J.l;
    double *X = fine_array(M, FX), *R = fine_array(M, FR), *Z = fine_array(M, FZ), *Q = fine_array(M, FQ);
    double* Pb[2] = {fine_array(M, FP), fine_array(M, FP2)};
    const Lv<double> F = fine_level(M);  // FP64 weights: stencil apply of CG
    Lv<double, float> FV;                // FP32 weights: the V-cycle
    FV.wx = reinterpret_cast<float*>(fine_array(M, FWX32));
    FV.wy = reinterpret_cast<float*>(fine_array(M, FWY32));
    FV.x = Z; FV.b = R; FV.kap = nullptr;
    FV.n = F.n; FV.lg = F.lg; FV.s = F.s;
    const int s = F.s;
    const double h2 = 1.0 / (double)(F.n * F.n);
    const double* kap = (const double*)J.kap;
    // WK = 2 instances run the fused row walks (their launch guarantees a
    // walked level, V(1,1) and the LDS ring); the new z goes to Q's array,
    // and the two swap after every cycle
    constexpr bool walks = WK == 2;
    zero_boundary<BS>(X, F.n);
    zero_boundary<BS>(Z, F.n);
    zero_boundary<BS>(Pb[0], F.n);
    zero_boundary<BS>(Pb[1], F.n);
    if (walks) zero_boundary<BS>(Q, F.n);
    setup_hierarchy<BS>(M, F, kap, FV.wx, FV.wy, walks);
    if (l == 2) build_coarse_inverse<BS>(FV, M.cinv);
    else if (l >= 3) build_coarse_inverse<BS>(coarse_level(M, 2), M.cinv);
    // The forward map needs the solution only at the observation points
    // unless the whole field is asked for (p_out; KEEP_X).  G = Obs x is
    // linear in x = sum_k alpha_k p_k, so without p_out each step adds
    // alpha_k Obs p_k to G as soon as alpha_k is known, and x is never
    // stored: the stencil pass then neither reads nor writes it (16 B less
    // per unknown and iteration).
    constexpr bool keep_x = KEEP_X;
    MLS_FOR_INTERIOR(F, {
        if (keep_x) X[c] = 0.0;
        R[c] = h2;
    })
    if (!keep_x)
        for (int o = threadIdx.x; o < C.nobs; o += BS) J.G[o] = 0.0;
    __syncthreads();
    if (walks) {
        vcycle_walk<BS>(M, FV, R, (const double*)nullptr, 0.0, (double*)nullptr, (const double*)nullptr, Z, Q,
                        false, red);
        double* t_ = Z; Z = Q; Q = t_;
    } else {
        vcycle<BS>(M, FV, R, Z, C.nu, false, false, red);
    }
    double rz = 0.0;
    MLS_FOR_INTERIOR(F, { rz += R[c] * Z[c]; })
    rz = block_sum<BS>(rz, red);
    const double rz0 = rz;
    int it = 0;
    int8_t st = 1;
    if (!(rz0 > 0.0) || !isfinite(rz0)) st = 2;
    // p_k = z_k + beta_k p_{k-1} (p_0 = z_0: beta = 0 with z as the old p)
    const double* Po = Z;
    double beta = 0.0;
    // x += alpha p is applied one iteration late, by the next stencil pass,
    // which reads that p at every node anyway; the last one after the loop
    double xa = 0.0;
    const double* Pl = nullptr;
    while (st == 1 && it < C.max_iters) {
        double* Pn = Pb[it & 1];
        // the p update and q = A p in one pass: the four neighbours' new p
        // are formed from z and the old p on the fly (bitwise the values
        // stored at those nodes), so the pass needs no barrier in between
        double pq = 0.0;
        auto pn = [&](int q) { return fma(beta, Po[q], Z[q]); };
        double* Xu = keep_x && it > 0 ? X : nullptr;
        if (WK >= 1 && F.n >= 64 && BS % F.n == 0) {
            pq = walk_apply<BS, WK == 2>(F, Z, Po, beta, Pn, Q, Xu, xa);
        } else {
            MLS_FOR_INTERIOR(F, {
                if (Xu) Xu[c] += xa * Po[c];
                const double pc = pn(c);
                const double v = diag_at(F.wx, F.wy, c, s) * pc
                               - (F.wx[c - 1] * pn(c - 1) + F.wx[c] * pn(c + 1) + F.wy[c - s] * pn(c - s)
                                  + F.wy[c] * pn(c + s));
                Pn[c] = pc;
                Q[c] = v;
                pq += pc * v;
            })
        }
        pq = block_sum<BS>(pq, red);
        const double alpha = rz / pq;
        xa = alpha;
        Pl = Pn;
        // Pn is complete (the reduction's barriers) and no pass writes it
        // before the next stencil pass
        if (!keep_x) observe_step<BS>(J, C, Pn, alpha);
        double rzn;
        if (walks) {  // the r update rides on the down walk
            rzn = vcycle_walk<BS>(M, FV, R, Q, alpha, (double*)nullptr, (const double*)nullptr, Z, Q, true, red);
            double* t_ = Z; Z = Q; Q = t_;
        } else {
            // the r update fused with the first red sweep of the V-cycle
            MLS_FOR_INTERIOR(F, {
                const double rn = R[c] - alpha * Q[c];
                R[c] = rn;
                Z[c] = (((i + j) & 1) == 0) ? rn / ldiag(FV, c) : 0.0;  // black: taken as zero
            })
            __syncthreads();
            rzn = vcycle<BS>(M, FV, R, Z, C.nu, l > 1, true, red);
        }
        ++it;
        if (!isfinite(rzn)) { st = 2; break; }
        if (rzn <= C.tol2 * rz0) { st = 0; break; }
        beta = rzn / rz;
        rz = rzn;
        Po = Pn;
    }
    if (Pl && keep_x) {  // the last pending x += alpha p
        MLS_FOR_INTERIOR(F, { X[c] += xa * Pl[c]; })
        __syncthreads();
    }
    observe_and_store<BS, keep_x>(J, C, X, F.n, st, it, red);
}

// --------------------------------------------------------- mixed solve --
// FP32 multigrid-PCG with residual replacement in FP64: the system matrix is
// the one defined by the FP32 edge weights (promoted exactly to FP64 for the
// residual).  The CG recurrence runs in FP32 on the correction x32 since the
// last replacement; whenever (r, z) has fallen by kDrift2 since then, x32 is
// folded into the FP64 iterate x64 and r is replaced by the FP64 residual
// b - A x64 rounded to FP32, and the recurrence goes on with the same search
// direction.  This bounds the drift between the recursive and the true
// residual without restarting CG, so the iteration count stays near the
// FP64 solver's.  Convergence is decided like the FP64 solver's, on the
// preconditioned norm (r, V r) relative to its first value, and confirmed
// on a freshly replaced residual.  The coarsest solve of the hierarchy is
// done in FP64.
constexpr double kDrift2 = 1e-6;  // replace r after (r, z) fell by this factor (1e-3 in norm)

template <int BS, int WK>
__device__ void solve_one_mixed(const Map<float>& M, const Job& J, const Common& C, double* red)
{
    const int l = J.l;
    float *X = fine_array(M, FX), *R = fine_array(M, FR), *Z = fine_array(M, FZ), *Q = fine_array(M, FQ);
    float* Pb[2] = {fine_array(M, FP), fine_array(M, FP2)};
    const Lv<float> F = fine_level(M);
    const int s = F.s;
    const int64_t hier = hier_elems(l, true);
    double* X64 = (double*)(M.slot + ((hier + 1) & ~int64_t(1)));
    const double h2 = 1.0 / (double)(F.n * F.n);
    const float* kap = (const float*)J.kap;
    constexpr bool walks = WK == 2;  // as in the FP64 solver
    zero_boundary<BS>(X, F.n);
    zero_boundary<BS>(Z, F.n);
    zero_boundary<BS>(Pb[0], F.n);
    zero_boundary<BS>(Pb[1], F.n);
    zero_boundary<BS>(X64, F.n);
    if (walks) zero_boundary<BS>(Q, F.n);
    setup_hierarchy<BS>(M, F, kap, nullptr, nullptr, walks);
    MLS_FOR_INTERIOR(F, { X64[c] = 0.0; X[c] = 0.f; R[c] = (float)h2; })
    __syncthreads();
    // x64 += x32, x32 = 0, then r = b - A x64 in FP64 (rounded to FP32)
    auto replace_residual = [&]() {
        MLS_FOR_INTERIOR(F, {
            X64[c] += (double)X[c];
            X[c] = 0.f;
        })
        __syncthreads();
        MLS_FOR_INTERIOR(F, {
            const double d = (double)F.wx[c - 1] + (double)F.wx[c] + (double)F.wy[c - s] + (double)F.wy[c];
            const double nb = (double)F.wx[c - 1] * X64[c - 1] + (double)F.wx[c] * X64[c + 1]
                            + (double)F.wy[c - s] * X64[c - s] + (double)F.wy[c] * X64[c + s];
            R[c] = (float)(h2 - (d * X64[c] - nb));
        })
        __syncthreads();
    };
    auto precondition = [&]() {  // z = V r and (r, z)
        if (walks) {
            const double d = vcycle_walk<BS>(M, F, R, (const float*)nullptr, 0.f, (float*)nullptr,
                                             (const float*)nullptr, Z, Q, true, red);
            float* t_ = Z; Z = Q; Q = t_;
            return d;
        }
        vcycle<BS>(M, F, R, Z, C.nu, false, false, red);
        double rz = 0.0;
        MLS_FOR_INTERIOR(F, { rz += (double)R[c] * (double)Z[c]; })
        return block_sum<BS>(rz, red);
    };
    double rz = precondition();
    const double rz0 = rz;
    int it = 0;
    int8_t st = 1;
    if (!(rz0 > 0.0) || !isfinite(rz0)) st = 2;
    double rz_upd = rz0;  // (r, z) at the last replacement
    // p_k = z_k + beta_k p_{k-1}, formed inside the stencil pass as in the
    // FP64 solver (p_0 = z_0 with beta = 0)
    const float* Po = Z;
    float beta = 0.f;
    while (st == 1 && it < C.max_iters) {
        float* Pn = Pb[it & 1];
        double pq = 0.0;
        auto pn = [&](int q) { return fmaf(beta, Po[q], Z[q]); };
        if (WK >= 1 && F.n >= 64 && BS % F.n == 0) {
            pq = walk_apply<BS, WK == 2>(F, Z, Po, beta, Pn, Q);
        } else {
            MLS_FOR_INTERIOR(F, {
                const float pc = pn(c);
                const float v = diag_at(F.wx, F.wy, c, s) * pc
                              - (F.wx[c - 1] * pn(c - 1) + F.wx[c] * pn(c + 1) + F.wy[c - s] * pn(c - s)
                                 + F.wy[c] * pn(c + s));
                Pn[c] = pc;
                Q[c] = v;
                pq += (double)pc * (double)v;
            })
        }
        pq = block_sum<BS>(pq, red);
        const float alpha = (float)(rz / pq);
        double rzn;
        if (walks) {  // the x and r updates ride on the down walk
            rzn = vcycle_walk<BS>(M, F, R, Q, alpha, X, Pn, Z, Q, true, red);
            float* t_ = Z; Z = Q; Q = t_;
        } else {
            MLS_FOR_INTERIOR(F, {
                X[c] += alpha * Pn[c];
                const float rn = R[c] - alpha * Q[c];
                R[c] = rn;
                Z[c] = (((i + j) & 1) == 0) ? rn / diag_at(F.wx, F.wy, c, s) : 0.f;  // black: taken as zero
            })
            __syncthreads();
            rzn = vcycle<BS>(M, F, R, Z, C.nu, l > 1, true, red);
        }
        ++it;
        if (!isfinite(rzn)) { st = 2; break; }
        const bool conv = rzn <= C.tol2 * rz0;
        if (conv || rzn <= kDrift2 * rz_upd) {
            replace_residual();
            if (conv) {  // confirm on the replaced residual
                const double rzt = precondition();
                if (!isfinite(rzt)) { st = 2; break; }
                if (rzt <= C.tol2 * rz0) { st = 0; break; }
                // not there yet: go on from the true residual, directions restarted
                rz = rzt;
                rz_upd = rzt;
                Po = Z;
                beta = 0.f;
                continue;
            }
            rz_upd = rzn;
        }
        beta = (float)(rzn / rz);
        rz = rzn;
        Po = Pn;
    }
    if (st != 0) {  // fold what the recurrence gathered since the last replacement
        MLS_FOR_INTERIOR(F, { X64[c] += (double)X[c]; })
        __syncthreads();
    }
    observe_and_store<BS>(J, C, X64, F.n, st, it, red);
}

// ----------------------------------------------------- single-level kernel --
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
    int64_t lds_elems;  // LDS budget in elements of the working type
    int cinv_lds;       // FP64: the coarse inverse follows the budget in LDS (else in the slot)
    int64_t ring_off;   // element offset of the row walks' LDS rows, or -1 (no walks)
    unsigned long long* queue;  // [0]: particles handed out, [1]: workgroups done; zero between launches
    Common C;
};

extern __shared__ __align__(16) char mls_lds[];

// FP64 solver kernels: ask for registers that leave room for six waves per
// SIMD (measured faster at h = 1/512 than the compiler's own choice, equal
// at h = 1/64); the FP32 kernels measured best unconstrained.  The
// column-walk instances run two 512-wide workgroups per CU at h = 1/512 and
// at the tuned h = 1/64 shape, which four waves per SIMD hold without
// spilling.
#define MLS_SOLVER_ATTR __attribute__((amdgpu_waves_per_eu(WK == 2 ? (MIXED ? 4 : 3) : (MIXED ? 1 : (WK ? 4 : 6)))))

// PX: the launch asks for the solution field (p_out), so the FP64 solve
// keeps its iterate; without it the FP64 solve gathers only the
// observations (separate instances: one kernel holding both variants
// spills heavily).  The mixed solve always keeps its FP64 iterate.
template <int BS, bool MIXED, int WK, bool PX>
__global__ __launch_bounds__(BS) MLS_SOLVER_ATTR void solve_kernel(SolveParams P)
{
    __shared__ double red[BS / 64];
    const int l = P.l;
    const int64_t ne = int64_t(2) << (2 * l);
    const int64_t M = ((int64_t(1) << l) - 1) * ((int64_t(1) << l) - 1);
    const int64_t NN = P.N_dev ? min(P.N, *P.N_dev) : P.N;
    // Particles are handed out one at a time from a counter in device
    // memory, so a workgroup that drew quick solves takes more of them and
    // the launch ends with the last particle, not with the unluckiest
    // workgroup's share.  The draw is broadcast through the reduction
    // array, which is free between particles.
    auto draw = [&]() -> int64_t {
        if (threadIdx.x == 0) *(int64_t*)red = (int64_t)atomicAdd(P.queue, 1ull);
        __syncthreads();
        const int64_t v = *(const int64_t*)red;
        __syncthreads();
        return v;
    };
    for (int64_t q = draw(); q < NN; q = draw()) {
        Job J;
        J.l = l;
        J.kap = MIXED ? (const void*)((const float*)P.kappa + q * ne) : (const void*)((const double*)P.kappa + q * ne);
        J.G = P.G + q * P.C.nobs;
        J.p_out = P.p_out ? P.p_out + q * M : nullptr;
        J.status = P.status ? P.status + q : nullptr;
        J.iters = P.iters ? P.iters + q : nullptr;
        J.y = P.y;
        J.phi = P.phi ? P.phi + q : nullptr;
        J.obs_idx = P.obs_idx;
        J.obs_w = P.obs_w;
        if (MIXED) {
            float* ring = (WK == 2 && P.ring_off >= 0) ? (float*)mls_lds + P.ring_off : nullptr;
            solve_one_mixed<BS, WK>(make_map((float*)P.ws + (int64_t)blockIdx.x * P.slot_elems, (float*)mls_lds, l,
                                         P.lds_elems, nullptr, ring), J, P.C, red);
        } else {
            double* slot = (double*)P.ws + (int64_t)blockIdx.x * P.slot_elems;
            double* cinv = P.cinv_lds ? (double*)mls_lds + P.lds_elems : slot + hier_elems(l, false);
            double* ring = (WK == 2 && P.ring_off >= 0) ? (double*)mls_lds + P.ring_off : nullptr;
            solve_one_f64<BS, WK, PX>(make_map(slot, (double*)mls_lds, l, P.lds_elems, cinv, ring), J, P.C, red);
        }
    }
    // every workgroup has drawn past the end; the last one to finish resets
    // the counter for the next launch on this context
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(P.queue + 1, 1ull) == (unsigned long long)(gridDim.x - 1)) {
            atomicExch(P.queue, 0ull);
            atomicExch(P.queue + 1, 0ull);
        }
    }
}

// -------------------------------------------------- work-list kernel --
// One persistent launch over the particles of many (instance, level)
// items: particle p belongs to the item whose prefix range holds p; items
// are ordered by level, finest first, so the costliest particles start
// first.  Slots are sized for the finest level in the list.
struct ListParams {
    const SolveItem* items;
    int n_items;
    int64_t total;
    void* ws;
    int64_t slot_elems;
    const int32_t* obs_idx[kMaxLevel + 1];
    const double* obs_w[kMaxLevel + 1];
    int64_t lds_elems;
    int cinv_lds;
    int64_t ring_off;
    Common C;
};

template <int BS, bool MIXED, int WK>
__global__ __launch_bounds__(BS) MLS_SOLVER_ATTR void solve_list_kernel(ListParams P)
{
    __shared__ double red[BS / 64];
    for (int64_t p = blockIdx.x; p < P.total; p += gridDim.x) {
        int lo = 0, hi = P.n_items - 1;  // last item with base <= p
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (P.items[mid].base <= p) lo = mid; else hi = mid - 1;
        }
        const SolveItem& it = P.items[lo];
        const int64_t q = p - it.base;
        const int l = it.l;
        const int64_t ne = int64_t(2) << (2 * l);
        Job J;
        J.l = l;
        J.kap = MIXED ? (const void*)((const float*)it.kappa + q * ne) : (const void*)((const double*)it.kappa + q * ne);
        J.G = it.G + q * P.C.nobs;
        J.p_out = nullptr;
        J.status = it.status ? it.status + q : nullptr;
        J.iters = it.iters ? it.iters + q : nullptr;
        J.y = it.y;
        J.phi = it.phi ? it.phi + q : nullptr;
        J.obs_idx = P.obs_idx[l];
        J.obs_w = P.obs_w[l];
        if (MIXED) {
            float* ring = (WK == 2 && P.ring_off >= 0) ? (float*)mls_lds + P.ring_off : nullptr;
            solve_one_mixed<BS, WK>(make_map((float*)P.ws + (int64_t)blockIdx.x * P.slot_elems, (float*)mls_lds, l,
                                         P.lds_elems, nullptr, ring), J, P.C, red);
        } else {
            double* slot = (double*)P.ws + (int64_t)blockIdx.x * P.slot_elems;
            double* cinv = P.cinv_lds ? (double*)mls_lds + P.lds_elems : slot + hier_elems(l, false);
            double* ring = (WK == 2 && P.ring_off >= 0) ? (double*)mls_lds + P.ring_off : nullptr;
            solve_one_f64<BS, WK, false>(make_map(slot, (double*)mls_lds, l, P.lds_elems, cinv, ring), J, P.C,
                                         red);  // work items carry no p_out
        }
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

static Common make_common(const mls2mc_ctx* ctx, int l)
{
    Common C;
    C.nobs = ctx->nobs;
    C.inv_sigma = 1.0 / ctx->prob.sigma_n;
    C.tol2 = ctx->rtol * ctx->rtol;
    C.max_iters = ctx->max_iters;
    C.nu = (l >= 0 && ctx->solver_nu[l] > 0) ? ctx->solver_nu[l] : 1;
    return C;
}

// solve_kernel instances: WK selects the column walk of the CG stencil pass
#define MLS_SWITCH_SOLVE(bs, MIXED, WK, PX, grid, lds, stream, params)                           \
    switch (bs) {                                                                                \
        case 64: solve_kernel<64, MIXED, WK, PX><<<grid, 64, lds, stream>>>(params); break;       \
        case 128: solve_kernel<128, MIXED, WK, PX><<<grid, 128, lds, stream>>>(params); break;    \
        case 256: solve_kernel<256, MIXED, WK, PX><<<grid, 256, lds, stream>>>(params); break;    \
        case 512: solve_kernel<512, MIXED, WK, PX><<<grid, 512, lds, stream>>>(params); break;    \
        case 1024: solve_kernel<1024, MIXED, WK, PX><<<grid, 1024, lds, stream>>>(params); break; \
        default: MLS_REQUIRE(false, "solver: unsupported block size");                           \
    }

// solve_list_kernel instances, WK as for solve_kernel (each item decides)
#define MLS_SWITCH_LIST(bs, MIXED, WK, grid, lds, stream, params)                                \
    switch (bs) {                                                                                \
        case 64: solve_list_kernel<64, MIXED, WK><<<grid, 64, lds, stream>>>(params); break;      \
        case 128: solve_list_kernel<128, MIXED, WK><<<grid, 128, lds, stream>>>(params); break;   \
        case 256: solve_list_kernel<256, MIXED, WK><<<grid, 256, lds, stream>>>(params); break;   \
        case 512: solve_list_kernel<512, MIXED, WK><<<grid, 512, lds, stream>>>(params); break;   \
        case 1024: solve_list_kernel<1024, MIXED, WK><<<grid, 1024, lds, stream>>>(params); break;\
        default: MLS_REQUIRE(false, "solver: unsupported block size");                           \
    }

// LDS bytes for level l under the level's budget (0 = no LDS residency).
// *alloc_elems is what the launch allocates; kernels decide each particle's
// residency with it as the budget, so no level uses more than is allocated
// (the policy is monotone in the budget).
// The FP64 kernels' coarse inverse goes after those elements when the
// budget has room for it (or there is no residency), else in the slot: the
// launch takes no more LDS than the budget (or than the inverse's 648 bytes
// under a smaller one), so the workgroups per CU that a budget was chosen
// for still fit.
static size_t lds_bytes_for(const mls2mc_ctx* ctx, int l, bool mixed, int bs, bool walks, int64_t* alloc_elems,
                            int* cinv_lds, int64_t* ring_off)
{
    const size_t esz = mixed ? sizeof(float) : sizeof(double);
    int64_t budget = ctx->solver_lds[l] >= 0 ? (ctx->solver_lds[l] ? ctx->solver_lds[l] : 65536) : 0;
    if (budget > ctx->max_lds) budget = ctx->max_lds;
    // the row walks' rows come first: the residency gets what is left
    const int64_t ring = walks ? walk_ring_elems(bs, l) : 0;
    const int64_t ring_bytes = ring * (int64_t)esz;
    const int64_t cinv_bytes = mixed ? 0 : kCinvElems * 8;
    if (walks && budget > ctx->max_lds - ring_bytes - cinv_bytes)
        budget = std::max<int64_t>(0, ctx->max_lds - ring_bytes - cinv_bytes);
    *alloc_elems = lds_elems_used(l, !mixed, (int64_t)(budget / esz));
    const int64_t room = budget > kCinvElems * 8 ? budget : kCinvElems * 8;
    *cinv_lds = !mixed && (walks || (*alloc_elems + kCinvElems) * 8 <= room);
    const int64_t off = *alloc_elems + (*cinv_lds ? kCinvElems : 0);
    *ring_off = walks ? off : -1;
    return (size_t)(off + ring) * esz;
}

// the fused row walks of the V-cycle run for V(1,1) from h = 1/256 on when
// half the row width divides the workgroup (walk_level)
static bool launch_walks(int l, int bs, int nu)
{
    return nu == 1 && l >= 8 && bs % (1 << (l - 1)) == 0;
}

int launch_solve(mls2mc_ctx* ctx, const SolveArgs& a, hipStream_t s)
{
    if (a.N == 0) return MLS2MC_OK;
    if (ctx->prob.bc == MLS2MC_BC_FLOW_CELL) return launch_flow_solve(ctx, a, s);
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
    P.obs_idx = ctx->obs[l].idx; P.obs_w = ctx->obs[l].w;
    P.queue = ctx->d_queue;
    P.C = make_common(ctx, l);
    const bool fused = launch_walks(l, bs, P.C.nu);
    const size_t lds = lds_bytes_for(ctx, l, mixed, bs, fused, &P.lds_elems, &P.cinv_lds, &P.ring_off);
    ProfRec rec;
    if (ctx->prof_on) {
        if (!P.iters) {  // the iteration totals need per-particle counts
            MLS_TRY(ctx->ws_prof.ensure(sizeof(int32_t) * (size_t)a.N));
            P.iters = ctx->ws_prof.as<int32_t>();
        }
        MLS_TRY(prof_begin(ctx, MLS2MC_PROF_SOLVE, l, a.N, s, &rec));
    }
    dim3 g((unsigned)grid);
    // from h = 1/64 on, when the row width divides the workgroup, the CG
    // stencil pass walks columns (measured faster from there; the smaller
    // levels are latency bound)
    const bool walk = l >= 6 && bs % (1 << l) == 0;
    const bool px = P.p_out != nullptr;
    if (fused) {
        if (mixed) { MLS_SWITCH_SOLVE(bs, true, 2, true, g, lds, s, P) }
        else if (px) { MLS_SWITCH_SOLVE(bs, false, 2, true, g, lds, s, P) }
        else { MLS_SWITCH_SOLVE(bs, false, 2, false, g, lds, s, P) }
    } else if (walk) {
        if (mixed) { MLS_SWITCH_SOLVE(bs, true, 1, true, g, lds, s, P) }
        else if (px) { MLS_SWITCH_SOLVE(bs, false, 1, true, g, lds, s, P) }
        else { MLS_SWITCH_SOLVE(bs, false, 1, false, g, lds, s, P) }
    } else {
        if (mixed) { MLS_SWITCH_SOLVE(bs, true, 0, true, g, lds, s, P) }
        else if (px) { MLS_SWITCH_SOLVE(bs, false, 0, true, g, lds, s, P) }
        else { MLS_SWITCH_SOLVE(bs, false, 0, false, g, lds, s, P) }
    }
    MLS_CHECK_HIP(hipGetLastError());
    if (ctx->prof_on) {
        MLS_TRY(prof_end(ctx, MLS2MC_PROF_SOLVE, l, rec, s));
        MLS_TRY(launch_reduce_i32(a.N, P.iters, nullptr, ctx->d_prof_iters + 2 * l, s));
    }
    return MLS2MC_OK;
}

// Work-list launch.  items_dev: device copy of the items (bases set, finest
// level first); lmax: finest level in the list; total: sum of N.
static void list_shape(const mls2mc_ctx* ctx, int lmax, int64_t total, bool mixed, int64_t* grid,
                       int64_t* slot, int* bs);

int launch_solve_list(mls2mc_ctx* ctx, const SolveItem* items_dev, int n_items, int64_t total, int lmax,
                      bool mixed, hipStream_t s)
{
    if (total == 0 || n_items == 0) return MLS2MC_OK;
    int64_t grid, slot;
    int bs;
    list_shape(ctx, lmax, total, mixed, &grid, &slot, &bs);
    const size_t esz = mixed ? sizeof(float) : sizeof(double);
    MLS_TRY(ctx->ws_solver.ensure((size_t)grid * slot * esz));
    ListParams P;
    P.items = items_dev;
    P.n_items = n_items;
    P.total = total;
    P.ws = ctx->ws_solver.ptr;
    P.slot_elems = slot;
    for (int l = 0; l <= kMaxLevel; ++l) {
        P.obs_idx[l] = ctx->obs[l].idx;
        P.obs_w[l] = ctx->obs[l].w;
    }
    P.C = make_common(ctx, lmax);
    // the work list mixes levels, so it keeps the separate V-cycle passes
    const size_t lds = lds_bytes_for(ctx, lmax, mixed, bs, false, &P.lds_elems, &P.cinv_lds, &P.ring_off);
    dim3 g((unsigned)grid);
    // items of h = 1/64 and finer walk columns in the CG stencil pass (the
    // instance decides per item)
    if (lmax >= 6) {
        if (mixed) { MLS_SWITCH_LIST(bs, true, 1, g, lds, s, P) }
        else { MLS_SWITCH_LIST(bs, false, 1, g, lds, s, P) }
    } else {
        if (mixed) { MLS_SWITCH_LIST(bs, true, 0, g, lds, s, P) }
        else { MLS_SWITCH_LIST(bs, false, 0, g, lds, s, P) }
    }
    MLS_CHECK_HIP(hipGetLastError());
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
        // the flow-cell layout has a ghost row below j = 0
        const int row0 = ctx->prob.bc == MLS2MC_BC_FLOW_CELL ? s : 0;
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
                for (int k = 0; k < 3; ++k) { idx[3 * o + k] = row0 + nodes[k]; w[3 * o + k] = wt[k]; }
            }
        MLS_CHECK_HIP(hipMalloc(&ctx->obs[l].idx, sizeof(int32_t) * idx.size()));
        MLS_CHECK_HIP(hipMalloc(&ctx->obs[l].w, sizeof(double) * w.size()));
        MLS_CHECK_HIP(hipMemcpy(ctx->obs[l].idx, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice));
        MLS_CHECK_HIP(hipMemcpy(ctx->obs[l].w, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice));
    }
    return MLS2MC_OK;
}

}  // namespace mls

namespace mls {

// Fused forward over many items (instances and levels): items are ordered
// finest level first and cut into chunks whose coefficient buffer fits the
// field workspace (8 GiB); each chunk is one grouped GEMM launch and one
// persistent work-list solver launch.  prepare_list stages the work lists
// (pinned host memory, asynchronous copy) and sizes every workspace the
// launches use; enqueue_list only launches, so it can be captured in a HIP
// graph and replayed while the prepared lists stay valid.
static void list_shape(const mls2mc_ctx* ctx, int lmax, int64_t total, bool mixed, int64_t* grid,
                       int64_t* slot, int* bs)
{
    int64_t sl = solver_slot_elems(lmax, mixed);
    sl = (sl + 63) & ~int64_t(63);
    const size_t esz = mixed ? sizeof(float) : sizeof(double);
    int64_t g = ctx->list_grid ? ctx->list_grid : (int64_t)ctx->n_cu * 4;
    const int64_t cap = (int64_t)((16ull << 30) / (sl * esz));
    if (g > cap) g = cap;
    if (g > total) g = total;
    if (g < 1) g = 1;
    *grid = g;
    *slot = sl;
    *bs = ctx->list_block ? ctx->list_block : default_block(lmax);
}

int prepare_list(mls2mc_ctx* ctx, const std::vector<FwdItem>& items_in, std::vector<ListChunk>& out,
                 hipStream_t s)
{
    out.clear();
    std::vector<FwdItem> items;
    for (const auto& it : items_in)
        if (it.N > 0) items.push_back(it);
    if (items.empty()) return MLS2MC_OK;
    std::stable_sort(items.begin(), items.end(), [](const FwdItem& a, const FwdItem& b) { return a.l > b.l; });
    const bool mixed = ctx->prob.precision == MLS2MC_MIXED;
    const size_t esz = mixed ? sizeof(float) : sizeof(double);
    const size_t cap_bytes = 8ull << 30;
    struct Piece { FwdItem it; int64_t off; };
    std::vector<std::vector<Piece>> chunks(1);
    size_t used = 0;
    for (const auto& it : items) {
        const size_t per = (size_t)n_elem(it.l) * esz;
        int64_t done = 0;
        while (done < it.N) {
            const int64_t fit = (int64_t)((cap_bytes - used) / per);
            if (fit <= 0) { chunks.emplace_back(); used = 0; continue; }
            const int64_t n = std::min(fit, it.N - done);
            FwdItem p = it;
            p.N = n;
            chunks.back().push_back({p, done});
            used += (size_t)n * per;
            done += n;
        }
    }
    size_t max_kap = 0, stage_bytes = 0;
    for (const auto& ch : chunks) {
        size_t b = 0;
        for (const auto& pc : ch) b += (size_t)pc.it.N * n_elem(pc.it.l) * esz;
        max_kap = std::max(max_kap, b);
        stage_bytes += ((ch.size() * (sizeof(GemmItem) + sizeof(SolveItem))) + 255) & ~size_t(255);
    }
    MLS_TRY(ctx->ws_kappa.ensure(max_kap));
    if (ctx->h_list_bytes < stage_bytes) {
        if (ctx->h_list) {
            if (ctx->h_list_ev) (void)hipEventSynchronize(ctx->h_list_ev);
            (void)hipHostFree(ctx->h_list);
        }
        ctx->h_list = nullptr;
        ctx->h_list_bytes = 0;
        MLS_CHECK_HIP(hipHostMalloc(&ctx->h_list, stage_bytes * 2));
        ctx->h_list_bytes = stage_bytes * 2;
    }
    MLS_TRY(ctx->ws_list.ensure(stage_bytes));
    // the previous call's asynchronous copies read the staging buffer
    if (ctx->h_list_ev) MLS_CHECK_HIP(hipEventSynchronize(ctx->h_list_ev));
    else MLS_CHECK_HIP(hipEventCreateWithFlags(&ctx->h_list_ev, hipEventDisableTiming));
    const int K = ctx->prob.K;
    char* hb = (char*)ctx->h_list;
    char* db = (char*)ctx->ws_list.ptr;
    size_t off = 0;
    size_t ws_need = 0;
    for (const auto& ch : chunks) {
        GemmItem* hg = (GemmItem*)(hb + off);
        SolveItem* hs = (SolveItem*)(hb + off + ch.size() * sizeof(GemmItem));
        ListChunk lc;
        lc.n = (int)ch.size();
        lc.tiles = 0;
        lc.total = 0;
        lc.lmax = 0;
        size_t kap_off = 0;
        for (size_t i = 0; i < ch.size(); ++i) {
            const FwdItem& it = ch[i].it;
            const int64_t q0 = ch[i].off;
            const int64_t ne = n_elem(it.l);
            void* kap = (char*)ctx->ws_kappa.ptr + kap_off;
            kap_off += (size_t)it.N * ne * esz;
            GemmItem g;
            g.theta = it.theta + q0 * K;
            g.B = ctx->d_B[it.l];
            g.B16 = ctx->d_B16[it.l];
            g.out = kap;
            g.N = it.N;
            g.ne = ne;
            g.tile_base = lc.tiles;
            g.tiles_x = (ne + 63) / 64;
            lc.tiles += g.tiles_x * ((it.N + 63) / 64);
            hg[i] = g;
            SolveItem v;
            v.l = it.l;
            v.N = it.N;
            v.base = lc.total;
            v.kappa = kap;
            v.G = it.G + q0 * ctx->nobs;
            v.phi = it.phi ? it.phi + q0 : nullptr;
            v.y = it.y;
            v.status = it.status ? it.status + q0 : nullptr;
            v.iters = it.iters ? it.iters + q0 : nullptr;
            hs[i] = v;
            lc.total += it.N;
            lc.lmax = std::max(lc.lmax, it.l);
        }
        const size_t bytes = ch.size() * (sizeof(GemmItem) + sizeof(SolveItem));
        MLS_CHECK_HIP(hipMemcpyAsync(db + off, hb + off, bytes, hipMemcpyHostToDevice, s));
        lc.gemm = (const GemmItem*)(db + off);
        lc.solve = (const SolveItem*)(db + off + ch.size() * sizeof(GemmItem));
        int64_t grid, slot;
        int bs;
        list_shape(ctx, lc.lmax, lc.total, mixed, &grid, &slot, &bs);
        ws_need = std::max(ws_need, (size_t)grid * slot * esz);
        out.push_back(lc);
        off += (bytes + 255) & ~size_t(255);
    }
    MLS_CHECK_HIP(hipEventRecord(ctx->h_list_ev, s));
    MLS_TRY(ctx->ws_solver.ensure(ws_need));
    return MLS2MC_OK;
}

int enqueue_list(mls2mc_ctx* ctx, const std::vector<ListChunk>& chunks, hipStream_t s)
{
    const bool mixed = ctx->prob.precision == MLS2MC_MIXED;
    for (const auto& lc : chunks) {
        MLS_TRY(launch_kl_list(ctx, lc.gemm, lc.n, lc.tiles, s));
        MLS_TRY(launch_solve_list(ctx, lc.solve, lc.n, lc.total, lc.lmax, mixed, s));
    }
    return MLS2MC_OK;
}

int forward_list(mls2mc_ctx* ctx, const std::vector<FwdItem>& items, hipStream_t s)
{
    MLS_REQUIRE(ctx->prob.bc == MLS2MC_BC_DIRICHLET, "batched forwards: Dirichlet problem only");
    std::vector<ListChunk> chunks;
    MLS_TRY(prepare_list(ctx, items, chunks, s));
    return enqueue_list(ctx, chunks, s);
}

}  // namespace mls

using namespace mls;

extern "C" int mls2mc_forward_batch(mls2mc_ctx* ctx, int n_items, const mls2mc_forward_item* items, void* stream)
{
    MLS_REQUIRE(ctx != nullptr, "null context");
    MLS_REQUIRE(n_items >= 0 && n_items <= 65536, "forward_batch: need 0 <= n_items <= 65536");
    MLS_REQUIRE(n_items == 0 || items, "forward_batch: null items");
    MLS_REQUIRE(!ctx->d_lin_A, "forward_batch: the linear test model runs through the single-instance entry points");
    std::vector<FwdItem> v;
    for (int i = 0; i < n_items; ++i) {
        const mls2mc_forward_item& it = items[i];
        MLS_REQUIRE(it.l >= ctx->prob.l_min && it.l <= ctx->prob.l_max, "forward_batch: level outside the context");
        MLS_REQUIRE(it.N >= 0, "forward_batch: N < 0");
        MLS_REQUIRE(it.N == 0 || (it.theta && it.G_out), "forward_batch: null pointer");
        MLS_REQUIRE(!it.phi_out || it.y, "forward_batch: phi_out needs y");
        v.push_back({it.l, it.N, it.theta, it.G_out, it.y, it.phi_out, it.status_out, it.iters_out});
    }
    return forward_list(ctx, v, (hipStream_t)stream);
}
