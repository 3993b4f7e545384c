// perrk_kernels.hip -- gfx950 kernels of one P-ERRK step (arXiv 2507.04991).
//
// Stage kernel: one wavefront of 64 lanes holds the nodes of one hexahedral
// element (3D, 4x4x4 LGL nodes) or of four quadrilateral elements (2D, 4x4
// nodes each); lane = node.  Each lane
//   1. forms its stage state U_{n,i} = U_n + dt ((c_i - a_{i,i-1}) K_1 + a_{i,i-1} K_{i-1})
//      with its level's coefficients (Sec. 2.2; inactive levels have a = 0,
//      the cheap update), in double precision;
//   2. converts it to primitive variables (and logarithms) and publishes them
//      in LDS;
//   3. accumulates, per direction, the flux-differencing volume term
//      sum_{m != i} Dsplit[i][m] f#(u_i, u_m) over the three other nodes of
//      its LGL line (Ranocha's EC/KEP flux) -- nonlinear, so plain VALU work;
//   4. on element faces forms the neighbour's stage state at the matching
//      node (with the neighbour's level coefficients) and adds the lifted
//      surface flux +-(1/q_boundary) f*(u-, u+); each element computes its own
//      faces from bit-identical arguments, so both sides see the same f*;
//   5. writes K_i = -sum_d (2/h_d) (...) in the stage storage precision, or,
//      in the last stage, the direction d = b_1 K_1 + b_{S-1} K_{S-1} + b_S K_S
//      in double precision;
//   6. if b_i != 0, reduces J q w(U_{n,i}) . K_i over the element's lanes
//      (fixed butterfly) into one partial per element (EntropyChange_...
//      rearranged node-wise form).
// Only the active prefix of the level-sorted element list is launched.
//
// Relaxation (Sec. 3.1): a residual pass reads U_n and d once per node and
// reduces J q [s(u + gamma dt d) - s(u)] (cancellation-free form),
// J q w(u + gamma dt d) . dt d and, when a bracket is being opened, the
// difference at a second point; one workgroup per case then sums the
// per-element partials in a fixed order and advances a Newton / bisection
// state machine held in device memory.  Per-element partials make every sum
// independent of the launch shape, so results are bitwise reproducible.

#include "perrk_internal.h"

#include <math.h>

namespace {

template <int DIM>
struct Geo {
    static constexpr int NPE = DIM == 2 ? 16 : 64;  // nodes per element
    static constexpr int V = DIM + 2;               // conserved fields
    static constexpr int EPW = 64 / NPE;            // elements per wavefront
    static constexpr int NQ = DIM + 5;              // LDS quantities per node
};

// Split-form SBP matrix of the degree-3 LGL rule, Dsplit = 2 D - W^-1 B,
// from closed forms (phi = (1 + sqrt 5) / 2):
//   D = [[-3, 5 phi/2, -5 (phi-1)/2, 1/2], [-phi/2, 0, sqrt5/2, -(phi-1)/2],
//        [(phi-1)/2, -sqrt5/2, 0, phi/2], [-1/2, 5 (phi-1)/2, -5 phi/2, 3]],
//   W = diag(1, 5, 5, 1)/6, B = diag(-1, 0, 0, 1).  Diagonal of Dsplit = 0.
#define PHI 1.61803398874989484820458683437
#define SQ5 2.23606797749978969640917366873
__constant__ double c_ds64[16] = {
    0.0, 5.0 * PHI, -5.0 * (PHI - 1.0), 1.0,
    -PHI, 0.0, SQ5, -(PHI - 1.0),
    PHI - 1.0, -SQ5, 0.0, PHI,
    -1.0, 5.0 * (PHI - 1.0), -5.0 * PHI, 0.0};
__constant__ float c_ds32[16] = {
    0.0f, (float)(5.0 * PHI), (float)(-5.0 * (PHI - 1.0)), 1.0f,
    (float)(-PHI), 0.0f, (float)SQ5, (float)(-(PHI - 1.0)),
    (float)(PHI - 1.0), (float)(-SQ5), 0.0f, (float)PHI,
    -1.0f, (float)(5.0 * (PHI - 1.0)), (float)(-5.0 * PHI), 0.0f};

template <typename T>
__device__ __forceinline__ T dsplit(int i, int m);
template <>
__device__ __forceinline__ double dsplit<double>(int i, int m) { return c_ds64[i * 4 + m]; }
template <>
__device__ __forceinline__ float dsplit<float>(int i, int m) { return c_ds32[i * 4 + m]; }

// 1D LGL weights: 1/6 at the ends, 5/6 inside.
__device__ __forceinline__ double lglw(int i) { return (i == 0 || i == 3) ? (1.0 / 6.0) : (5.0 / 6.0); }

template <int DIM>
__device__ __forceinline__ double node_weight(int node)
{
    double w = lglw(node & 3) * lglw((node >> 2) & 3);
    if (DIM == 3) w *= lglw(node >> 4);
    return w;
}

// ---------------------------------------------------------------- log mean
// (a - b) / (log a - log b).  Near a = b: with u = ((a-b)/(a+b))^2 the mean is
// (a+b) / (2 + 2u/3 + 2u^2/5 + ...), used for u < 1e-2 (truncated after u^8 in
// double, after u^3 in single precision: below the rounding unit).  Otherwise
// (a - b) / log(a/b): in double from the per-node logarithms, in single
// precision with the hardware logarithm of the ratio.
__device__ __forceinline__ double lmean(double a, double b, double la, double lb)
{
    const double d = a - b, s = a + b;
    const double d2 = d * d, s2 = s * s;
    if (d2 < 1.0e-2 * s2) {
        const double u = d2 / s2;
        const double F = 2.0 + u * (2.0 / 3.0 + u * (2.0 / 5.0 + u * (2.0 / 7.0 + u * (2.0 / 9.0 +
                         u * (2.0 / 11.0 + u * (2.0 / 13.0 + u * (2.0 / 15.0 + u * (2.0 / 17.0))))))));
        return s / F;
    }
    return d / (la - lb);
}

__device__ __forceinline__ float lmean(float a, float b, float, float)
{
    const float d = a - b, s = a + b;
    const float d2 = d * d, s2 = s * s;
    if (d2 < 1.0e-2f * s2) {
        const float u = d2 / s2;
        const float F = 2.0f + u * (2.0f / 3.0f + u * (2.0f / 5.0f + u * (2.0f / 7.0f)));
        return s / F;
    }
    return d / __logf(a / b);
}

// ---------------------------------------------------------------- node data
template <typename T, int DIM>
struct Prim {
    T rho, v[DIM], p, beta, lr, lb;  // beta = rho / p; lr, lb = logs (double path only)
};

// Primitive variables of a double-precision state.  Sets bit 1 of bad for
// rho <= 0 or p <= 0, bit 2 for non-finite input.
template <typename T, int DIM>
__device__ __forceinline__ void make_prim(const double *u, double gam, Prim<T, DIM> &P, int &bad)
{
    const double rho = u[0];
    const double ir = 1.0 / rho;
    double ke = 0.0;
    double v[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        v[k] = u[1 + k] * ir;
        ke += u[1 + k] * v[k];
    }
    const double p = (gam - 1.0) * (u[DIM + 1] - 0.5 * ke);
    bool fin = true;
#pragma unroll
    for (int k = 0; k < DIM + 2; ++k) fin = fin && isfinite(u[k]);
    if (!fin) bad |= 2;
    else if (!(rho > 0.0) || !(p > 0.0)) bad |= 1;
    P.rho = (T)rho;
#pragma unroll
    for (int k = 0; k < DIM; ++k) P.v[k] = (T)v[k];
    P.p = (T)p;
    if constexpr (sizeof(T) == 8) {
        P.beta = rho / p;
        P.lr = log(rho);
        P.lb = log(P.beta);
    } else {
        P.beta = (T)(rho / p);
        P.lr = 0;
        P.lb = 0;
    }
}

// Ranocha's entropy-conservative, kinetic-energy-preserving two-point flux in
// direction D: f_rho = {rho}_log {v_D}, f_m = f_rho {v} + {p} e_D,
// f_E = f_rho (v_L.v_R / 2 + 1 / ((gamma-1) {rho/p}_log)) + (p_L v_R,D + p_R v_L,D) / 2.
template <int D, typename T, int DIM>
__device__ __forceinline__ void flux_ec(const Prim<T, DIM> &L, const Prim<T, DIM> &R, T inv_gm1,
                                        T *f)
{
    const T rm = lmean(L.rho, R.rho, L.lr, R.lr);
    const T bm = lmean(L.beta, R.beta, L.lb, R.lb);
    const T fr = rm * (T)0.5 * (L.v[D] + R.v[D]);
    T vv = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) vv += L.v[k] * R.v[k];
    f[0] = fr;
#pragma unroll
    for (int k = 0; k < DIM; ++k) f[1 + k] = fr * (T)0.5 * (L.v[k] + R.v[k]);
    f[1 + D] += (T)0.5 * (L.p + R.p);
    f[DIM + 1] = fr * ((T)0.5 * vv + inv_gm1 / bm) + (T)0.5 * (L.p * R.v[D] + R.p * L.v[D]);
}

// HLL two-wave flux with Davis wave-speed estimates in direction D.
template <int D, typename T, int DIM>
__device__ __forceinline__ void flux_hll(const Prim<T, DIM> &L, const Prim<T, DIM> &R,
                                         const T *uL, const T *uR, T gam, T *f)
{
    const T cl = sqrt(gam * L.p / L.rho), cr = sqrt(gam * R.p / R.rho);
    const T lmin = fmin(L.v[D] - cl, R.v[D] - cr);
    const T lmax = fmax(L.v[D] + cl, R.v[D] + cr);
    T fl[DIM + 2], fr[DIM + 2];
    fl[0] = uL[0] * L.v[D];
    fr[0] = uR[0] * R.v[D];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        fl[1 + k] = uL[1 + k] * L.v[D];
        fr[1 + k] = uR[1 + k] * R.v[D];
    }
    fl[1 + D] += L.p;
    fr[1 + D] += R.p;
    fl[DIM + 1] = (uL[DIM + 1] + L.p) * L.v[D];
    fr[DIM + 1] = (uR[DIM + 1] + R.p) * R.v[D];
    if (lmin >= (T)0) {
#pragma unroll
        for (int k = 0; k < DIM + 2; ++k) f[k] = fl[k];
    } else if (lmax <= (T)0) {
#pragma unroll
        for (int k = 0; k < DIM + 2; ++k) f[k] = fr[k];
    } else {
        const T inv = (T)1 / (lmax - lmin);
#pragma unroll
        for (int k = 0; k < DIM + 2; ++k)
            f[k] = (lmax * fl[k] - lmin * fr[k] + lmin * lmax * (uR[k] - uL[k])) * inv;
    }
}

// Entropy variables of s = -rho log(p rho^-gamma):
// w = (gamma - log(p rho^-gamma) - (gamma-1) rho |v|^2 / (2p), (gamma-1) rho v / p, -(gamma-1) rho / p).
template <int DIM>
__device__ __forceinline__ void entropy_vars(const double *u, double gam, double *w)
{
    const double rho = u[0];
    const double ir = 1.0 / rho;
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) m2 += u[1 + k] * u[1 + k];
    const double p = (gam - 1.0) * (u[DIM + 1] - 0.5 * m2 * ir);
    const double rp = rho / p;
    const double g1rp = (gam - 1.0) * rp;
    w[0] = gam - (log(p) - gam * log(rho)) - 0.5 * g1rp * m2 * ir * ir;
#pragma unroll
    for (int k = 0; k < DIM; ++k) w[1 + k] = g1rp * u[1 + k] * ir;
    w[DIM + 1] = -g1rp;
}

// s(u) = -rho (log p - gamma log rho).
template <int DIM>
__device__ __forceinline__ double entropy_density(const double *u, double gam)
{
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) m2 += u[1 + k] * u[1 + k];
    const double p = (gam - 1.0) * (u[DIM + 1] - 0.5 * m2 / u[0]);
    return -u[0] * (log(p) - gam * log(u[0]));
}

// s(u + du) - s(u) without cancellation: with rho' = rho + drho,
// dp = (gamma-1) [dE - (m.dm + |dm|^2/2) / rho' + drho |m|^2 / (2 rho rho')] = p' - p and
// s' - s = -drho (log p' - gamma log rho') - rho [log1p(dp/p) - gamma log1p(drho/rho)].
template <int DIM>
__device__ __forceinline__ double entropy_diff(const double *u, const double *du, double gam)
{
    const double rho = u[0], drho = du[0], rho1 = rho + drho;
    double mdm = 0.0, dm2 = 0.0, m2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        mdm += u[1 + k] * du[1 + k];
        dm2 += du[1 + k] * du[1 + k];
        m2 += u[1 + k] * u[1 + k];
    }
    const double p = (gam - 1.0) * (u[DIM + 1] - 0.5 * m2 / rho);
    const double dp = (gam - 1.0) * (du[DIM + 1] - (mdm + 0.5 * dm2) / rho1 + drho * m2 / (2.0 * rho * rho1));
    const double p1 = p + dp;
    return -drho * (log(p1) - gam * log(rho1)) - rho * (log1p(dp / p) - gam * log1p(drho / rho));
}

template <typename T>
__device__ __forceinline__ T ld(const void *p, size_t i) { return static_cast<const T *>(p)[i]; }

// U_{n,i} at one node of element e: U_n + dt (c1 K_1 + cp K_{i-1}); K_{i-1} is
// read only when its coefficient is nonzero (it may hold stale data otherwise).
template <int DIM, typename KT, int KIND>
__device__ __forceinline__ void form_state(const StageArgs &a, const double *coef, int e, int node,
                                           int level, int case_id, double *u)
{
    constexpr int NPE = Geo<DIM>::NPE, V = Geo<DIM>::V;
    double dt = 0.0, c1 = 0.0, cp = 0.0;
    if (KIND != SK_FIRST) {
        dt = a.cs[case_id].dt;
        c1 = coef[level];
        cp = coef[PERRK_MAXR + level];
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const size_t idx = ((size_t)v * a.nelem + e) * NPE + node;
        double x = a.U[idx];
        if (KIND != SK_FIRST) {
            double s = c1 * (double)ld<KT>(a.K1, idx);
            if (cp != 0.0) s += cp * (double)ld<KT>(a.Kp, idx);
            x = x + dt * s;
        }
        u[v] = x;
    }
}

template <typename T, int DIM>
__device__ __forceinline__ void put_prim(T *sq, int eslot, int node, const Prim<T, DIM> &P)
{
    constexpr int NPE = Geo<DIM>::NPE, NQ = Geo<DIM>::NQ;
    T *b = sq + (size_t)eslot * NQ * NPE + node;
    b[0] = P.rho;
#pragma unroll
    for (int k = 0; k < DIM; ++k) b[(1 + k) * NPE] = P.v[k];
    b[(DIM + 1) * NPE] = P.p;
    b[(DIM + 2) * NPE] = P.beta;
    b[(DIM + 3) * NPE] = P.lr;
    b[(DIM + 4) * NPE] = P.lb;
}

template <typename T, int DIM>
__device__ __forceinline__ void get_prim(const T *sq, int eslot, int node, Prim<T, DIM> &P)
{
    constexpr int NPE = Geo<DIM>::NPE, NQ = Geo<DIM>::NQ;
    const T *b = sq + (size_t)eslot * NQ * NPE + node;
    P.rho = b[0];
#pragma unroll
    for (int k = 0; k < DIM; ++k) P.v[k] = b[(1 + k) * NPE];
    P.p = b[(DIM + 1) * NPE];
    P.beta = b[(DIM + 2) * NPE];
    P.lr = b[(DIM + 3) * NPE];
    P.lb = b[(DIM + 4) * NPE];
}

// One direction of the element operator at one node: volume flux differencing
// along the node's line plus the lifted surface flux on faces.
template <int D, int DIM, typename T, typename KT, int FLUX, int KIND>
__device__ __forceinline__ void direction_terms(const StageArgs &a, const double *coef, const T *sq,
                                                int eslot, int node, const ElemInfo &ei,
                                                const Prim<T, DIM> &me, const double *u, T *du,
                                                int &bad)
{
    constexpr int V = Geo<DIM>::V;
    constexpr int stride = D == 0 ? 1 : (D == 1 ? 4 : 16);
    const T inv_gm1 = (T)(1.0 / (a.gam - 1.0));
    const int id = (node / stride) & 3;
    T acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0;
#pragma unroll
    for (int j = 1; j < 4; ++j) {
        const int m = (id + j) & 3;
        Prim<T, DIM> P;
        get_prim<T, DIM>(sq, eslot, node + (m - id) * stride, P);
        T f[V];
        flux_ec<D, T, DIM>(me, P, inv_gm1, f);
        const T w = dsplit<T>(id, m);
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] += w * f[v];
    }
    if (id == 0 || id == 3) {
        const bool right = (id == 3);
        const int nb = ei.nbr[2 * D + (right ? 1 : 0)];
        const int nn = node + (right ? -3 : 3) * stride;
        const ElemInfo en = a.elem[nb];
        double un[V];
        form_state<DIM, KT, KIND>(a, coef, nb, nn, en.level, en.case_id, un);
        Prim<T, DIM> PN;
        make_prim<T, DIM>(un, a.gam, PN, bad);
        T f[V];
        if (FLUX == PERRK_FLUX_HLL) {
            T ul[V], ur[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                ul[v] = (T)(right ? u[v] : un[v]);
                ur[v] = (T)(right ? un[v] : u[v]);
            }
            if (right) flux_hll<D, T, DIM>(me, PN, ul, ur, (T)a.gam, f);
            else flux_hll<D, T, DIM>(PN, me, ul, ur, (T)a.gam, f);
        } else {
            if (right) flux_ec<D, T, DIM>(me, PN, inv_gm1, f);
            else flux_ec<D, T, DIM>(PN, me, inv_gm1, f);
        }
        const T lift = right ? (T)6 : (T)-6;  // +-1/q_boundary, q_boundary = 1/6
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] += lift * f[v];
    }
    const T h = (T)ei.metric[D];
#pragma unroll
    for (int v = 0; v < V; ++v) du[v] += h * acc[v];
}

}  // namespace

namespace {

template <int DIM, typename T, typename KT, int FLUX, int KIND>
__global__ void __launch_bounds__(256) stage_kernel(const StageArgs a, const double *coef)
{
    constexpr int NPE = Geo<DIM>::NPE, V = Geo<DIM>::V, EPW = Geo<DIM>::EPW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sq = reinterpret_cast<T *>(smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int eslot = wave * EPW + lane / NPE;
    const int node = lane % NPE;
    const int epb = (int)(blockDim.x >> 6) * EPW;
    const int li = blockIdx.x * epb + eslot;
    const bool valid = li < a.n_active;
    const int e = a.active[valid ? li : a.n_active - 1];
    const ElemInfo ei = a.elem[e];
    int bad = 0;

    double u[V];
    form_state<DIM, KT, KIND>(a, coef, e, node, ei.level, ei.case_id, u);
    Prim<T, DIM> me;
    make_prim<T, DIM>(u, a.gam, me, bad);
    put_prim<T, DIM>(sq, eslot, node, me);
    __syncthreads();

    T du[V];
#pragma unroll
    for (int v = 0; v < V; ++v) du[v] = 0;
    direction_terms<0, DIM, T, KT, FLUX, KIND>(a, coef, sq, eslot, node, ei, me, u, du, bad);
    direction_terms<1, DIM, T, KT, FLUX, KIND>(a, coef, sq, eslot, node, ei, me, u, du, bad);
    if constexpr (DIM == 3)
        direction_terms<2, DIM, T, KT, FLUX, KIND>(a, coef, sq, eslot, node, ei, me, u, du, bad);

    // K_i rounded to the stage storage precision
    double k[V];
#pragma unroll
    for (int v = 0; v < V; ++v) k[v] = (double)(KT)(-du[v]);

    if (valid) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const size_t idx = ((size_t)v * a.nelem + e) * NPE + node;
            if (KIND == SK_LAST) {
                double dv = a.bs * k[v];
                if (a.bsm1 != 0.0) dv += a.bsm1 * (double)ld<KT>(a.Kp, idx);
                if (a.b1 != 0.0) dv += a.b1 * (double)ld<KT>(a.K1, idx);
                a.d_out[idx] = dv;
            } else {
                static_cast<KT *>(a.Kout)[idx] = (KT)k[v];
            }
        }
    }
    if (a.ep_partial != nullptr) {
        double w[V];
        entropy_vars<DIM>(u, a.gam, w);
        double dot = 0.0;
#pragma unroll
        for (int v = 0; v < V; ++v) dot += w[v] * k[v];
        double s = node_weight<DIM>(node) * dot;
#pragma unroll
        for (int off = NPE / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off);
        if (valid && node == 0) a.ep_partial[e] = ei.jac * s;
    }
    if (bad && valid) atomicOr(a.err, bad);
}

// ---------------------------------------------------------------- reductions
// Sum of NC per-element partials over [b, e) by PERRK_RED_THREADS threads in a
// fixed order (strided sequential sums, then a fixed tree).  Result in out on
// every thread.
template <int NC>
__device__ __forceinline__ void case_sum(const double *part, int stride, int64_t b, int64_t e,
                                         double *out)
{
    __shared__ double red[NC][PERRK_RED_THREADS];
    const int t = threadIdx.x;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    for (int64_t i = b + t; i < e; i += PERRK_RED_THREADS) {
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += part[(size_t)i * stride + c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) red[c][t] = acc[c];
    __syncthreads();
    for (int h = PERRK_RED_THREADS / 2; h >= 1; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int c = 0; c < NC; ++c) red[c][t] += red[c][t + h];
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = red[c][0];
    __syncthreads();
}

// Per-element residual partials: J sum q Delta s at gamma, J sum q w(u + gamma dt d) . dt d,
// J sum q Delta s at gamma_b (only while opening a bracket), sum |d|.
template <int DIM>
__device__ __forceinline__ void relax_element(const double *U, const double *dd, const ElemInfo *elem,
                                              const CaseState *cs, double *partial, int64_t nelem,
                                              double gam, int64_t e, int node, bool valid)
{
    constexpr int NPE = Geo<DIM>::NPE, V = Geo<DIM>::V;
    const ElemInfo ei = elem[e];
    const CaseState &C = cs[ei.case_id];
    const int st = C.state;
    const bool live = valid && st != RS_DONE && st != RS_FALLBACK && st != RS_EVAL1;
    const bool eval1 = valid && st == RS_EVAL1;
    double sr = 0.0, srp = 0.0, srb = 0.0, sabs = 0.0;
    if (live || eval1) {
        const double g = eval1 ? 1.0 : C.gamma;
        const double dt = C.dt;
        double u[V], dv[V], du[V], u1[V], w[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const size_t idx = ((size_t)v * nelem + e) * NPE + node;
            u[v] = U[idx];
            dv[v] = dd[idx];
            du[v] = g * dt * dv[v];
            u1[v] = u[v] + du[v];
            sabs += fabs(dv[v]);
        }
        const double q = node_weight<DIM>(node);
        sr = q * entropy_diff<DIM>(u, du, gam);
        entropy_vars<DIM>(u1, gam, w);
        double dot = 0.0;
#pragma unroll
        for (int v = 0; v < V; ++v) dot += w[v] * dt * dv[v];
        srp = q * dot;
        if (!eval1 && st == RS_BIS_INIT) {
            const double gb = C.gamma_b;
#pragma unroll
            for (int v = 0; v < V; ++v) du[v] = gb * dt * dv[v];
            srb = q * entropy_diff<DIM>(u, du, gam);
        }
    }
#pragma unroll
    for (int off = NPE / 2; off >= 1; off >>= 1) {
        sr += __shfl_xor(sr, off);
        srp += __shfl_xor(srp, off);
        srb += __shfl_xor(srb, off);
        sabs += __shfl_xor(sabs, off);
    }
    if ((live || eval1) && node == 0) {
        double *pp = partial + (size_t)e * 4;
        pp[0] = ei.jac * sr;
        pp[1] = ei.jac * srp;
        pp[2] = ei.jac * srb;
        pp[3] = sabs;
    }
}

}  // namespace

namespace {

// Newton / bisection state machine of one case after a residual evaluation
// S = (sum Delta s at gamma, sum w . dt d at gamma, sum Delta s at gamma_b, sum |d|).
__device__ void relax_update(CaseState &C, const double *S, const RelaxParams &rp)
{
    const double off = (rp.anchor == 1) ? C.offset : 0.0;
    const int st = C.state;
    if (C.passes == 0 && S[3] == 0.0) {
        // d == 0 at the first evaluation: every gamma is a root
        C.state = RS_DONE;
        C.gamma_acc = 1.0;
        C.flags = PERRK_FLAG_TRIVIAL;
        C.r = off;
        C.H_delta = 0.0;
        return;
    }
    if (st == RS_NEWTON || st == RS_NEWTON_LAST) {
        const double r = S[0] - C.gamma * C.dH + off;
        const double rpv = S[1] - C.dH;
        C.passes += 1;
        C.r = r;
        C.rp = rpv;
        if (isfinite(r) && fabs(r) <= rp.tol_r) {
            C.state = RS_DONE;
            C.gamma_acc = C.gamma;
            C.H_delta = S[0];
            return;
        }
        bool to_bis = (st == RS_NEWTON_LAST) || !isfinite(r) || !isfinite(rpv) || rpv == 0.0;
        if (!to_bis) {
            const double step = r / rpv;
            C.gamma -= step;
            C.iters += 1;
            C.k += 1;
            if (!(C.gamma > 0.0)) to_bis = true;
            else if (fabs(step) < rp.tol_step) C.state = RS_NEWTON_LAST;
            else if (C.k >= rp.max_newton) to_bis = true;
        }
        if (to_bis) {
            C.state = RS_BIS_INIT;
            C.flags |= PERRK_FLAG_BISECT;
            C.widen = 0;
            C.gamma = rp.bis_lo;
            C.gamma_b = rp.bis_hi;
        }
        return;
    }
    if (st == RS_BIS_INIT) {
        const double ra = S[0] - C.gamma * C.dH + off;
        const double rb = S[2] - C.gamma_b * C.dH + off;
        C.passes += 2;
        if (isfinite(ra) && isfinite(rb) && ra < 0.0 && rb > 0.0) {
            C.state = RS_BIS;
            C.lo = C.gamma;
            C.hi = C.gamma_b;
            C.bis_count = 0;
            C.gamma = 0.5 * (C.lo + C.hi);
            if (rp.max_bisect <= 0) {
                C.state = RS_FALLBACK;
            }
        } else if (C.widen == 0) {
            C.widen = 1;
            C.gamma = 0.5 * rp.bis_lo;
            C.gamma_b = 2.0 * rp.bis_hi;
        } else {
            C.state = RS_FALLBACK;
        }
        return;
    }
    if (st == RS_BIS) {
        const double r = S[0] - C.gamma * C.dH + off;
        C.passes += 1;
        C.r = r;
        if (isfinite(r) && fabs(r) <= rp.tol_r) {
            C.state = RS_DONE;
            C.gamma_acc = C.gamma;
            C.H_delta = S[0];
            return;
        }
        if (r < 0.0) C.lo = C.gamma;
        else C.hi = C.gamma;
        C.bis_count += 1;
        if (C.bis_count >= rp.max_bisect) C.state = RS_FALLBACK;
        else C.gamma = 0.5 * (C.lo + C.hi);
    }
}

__global__ void __launch_bounds__(PERRK_RED_THREADS)
relax_prepare_kernel(CaseState *cs, const int64_t *case_off, const double *ep, int64_t nelem,
                     RelaxParams rp, const float *mlp)
{
    const int c = blockIdx.x;
    const int64_t b = case_off[c], e = case_off[c + 1];
    double ej[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < rp.nb; ++j) {
        double o[1];
        case_sum<1>(ep + (size_t)j * nelem, 1, b, e, o);
        ej[j] = o[0];
    }
    if (threadIdx.x != 0) return;
    CaseState &C = cs[c];
    double dH = 0.0;
    for (int j = 0; j < rp.nb; ++j) {
        C.e[j] = ej[j];
        dH += rp.bw[j] * ej[j];
    }
    C.dH = C.dt * dH;
    C.k = 0;
    C.iters = 0;
    C.passes = 0;
    C.flags = 0;
    C.bis_count = 0;
    C.widen = 0;
    C.r = 0.0;
    C.rp = 0.0;
    double g0 = C.gamma_prev;
    if (rp.guess == 1 && mlp != nullptr) {
        // learned guess of gamma - 1 (MLP 8-32-32-1, tanh), weights then mean[8], scale[8], out scale
        float x[8];
        x[0] = (float)C.ghist[0];
        x[1] = (float)C.ghist[1];
        x[2] = (float)C.ghist[2];
        x[3] = (float)C.dt;
        double sabs = 0.0;
        for (int j = 0; j < rp.nb; ++j) sabs += fabs(ej[j]);
        for (int j = 0; j < 4; ++j) x[4 + j] = (j < rp.nb && sabs > 0.0) ? (float)(ej[j] / sabs) : 0.0f;
        const float *W1 = mlp, *b1 = W1 + 256, *W2 = b1 + 32, *b2 = W2 + 1024, *W3 = b2 + 32, *b3 = W3 + 32;
        const float *mean = b3 + 1, *scale = mean + 8, *oscale = scale + 8;
        for (int i = 0; i < 8; ++i) x[i] = (x[i] - mean[i]) * scale[i];
        float h1[32], h2[32];
        for (int o = 0; o < 32; ++o) {
            float s = b1[o];
            for (int i = 0; i < 8; ++i) s += W1[o * 8 + i] * x[i];
            h1[o] = tanhf(s);
        }
        for (int o = 0; o < 32; ++o) {
            float s = b2[o];
            for (int i = 0; i < 32; ++i) s += W2[o * 32 + i] * h1[i];
            h2[o] = tanhf(s);
        }
        float y = b3[0];
        for (int i = 0; i < 32; ++i) y += W3[i] * h2[i];
        const double pred = (double)y * (double)oscale[0] + (double)oscale[1];
        if (isfinite(pred) && fabs(pred) < 0.5) g0 = 1.0 + pred;
    }
    C.gamma = g0;
    C.gamma_b = g0;
    C.H_delta = 0.0;
    C.state = rp.relax ? RS_NEWTON : RS_EVAL1;
    if (rp.relax && rp.max_newton <= 0) {  // no Newton budget: open the bracket at once
        C.state = RS_BIS_INIT;
        C.flags |= PERRK_FLAG_BISECT;
        C.gamma = rp.bis_lo;
        C.gamma_b = rp.bis_hi;
    }
    C.gamma_acc = 1.0;
}

template <int DIM>
__global__ void __launch_bounds__(256)
relax_pass_kernel(const double *U, const double *d, const ElemInfo *elem, const CaseState *cs,
                  double *partial, int64_t nelem, double gam)
{
    constexpr int NPE = Geo<DIM>::NPE, EPW = Geo<DIM>::EPW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t e0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * EPW + lane / NPE;
    const bool valid = e0 < nelem;
    relax_element<DIM>(U, d, elem, cs, partial, nelem, gam, valid ? e0 : nelem - 1, lane % NPE, valid);
}

__global__ void __launch_bounds__(PERRK_RED_THREADS)
relax_finalize_kernel(CaseState *cs, const int64_t *case_off, const double *partial, RelaxParams rp)
{
    const int c = blockIdx.x;
    const int st = cs[c].state;
    if (st == RS_DONE || st == RS_FALLBACK || st == RS_EVAL1) return;
    double S[4];
    case_sum<4>(partial, 4, case_off[c], case_off[c + 1], S);
    if (threadIdx.x == 0) relax_update(cs[c], S, rp);
}

// Runs the remaining residual evaluations of each case inside one workgroup
// (rarely needed: Newton usually converges within the launched passes), then
// the per-step bookkeeping.  Every evaluation uses the same per-element code and
// the same fixed-order sum as the launched passes.
template <int DIM>
__global__ void __launch_bounds__(PERRK_RED_THREADS)
relax_complete_kernel(const double *U, const double *d, const ElemInfo *elem, CaseState *cs,
                      const int64_t *case_off, double *partial, int64_t nelem, double gam,
                      RelaxParams rp)
{
    constexpr int NPE = Geo<DIM>::NPE, EPW = Geo<DIM>::EPW;
    const int c = blockIdx.x;
    const int64_t b = case_off[c], e = case_off[c + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = PERRK_RED_THREADS / 64;
    __shared__ int s_state;
    // bounded: Newton (+1), two bracket openings, bisection, one evaluation at gamma = 1
    const int max_iter = rp.max_newton + 4 + rp.max_bisect + 2;
    for (int it = 0; it <= max_iter; ++it) {
        if (threadIdx.x == 0) s_state = cs[c].state;
        __syncthreads();
        const int st = s_state;
        __syncthreads();
        if (st == RS_DONE) break;
        const bool one = (st == RS_FALLBACK || st == RS_EVAL1);
        if (one && threadIdx.x == 0) cs[c].state = RS_EVAL1;
        __syncthreads();
        for (int64_t g = b + (int64_t)wave * EPW; g < e; g += (int64_t)NW * EPW) {
            const int64_t el = g + lane / NPE;
            const bool valid = el < e;
            relax_element<DIM>(U, d, elem, cs, partial, nelem, gam, valid ? el : e - 1, lane % NPE,
                               valid);
        }
        __syncthreads();
        double S[4];
        case_sum<4>(partial, 4, b, e, S);
        if (threadIdx.x == 0) {
            CaseState &C = cs[c];
            if (one) {
                const double off = (rp.anchor == 1) ? C.offset : 0.0;
                C.gamma_acc = 1.0;
                C.H_delta = S[0];
                C.r = S[0] - C.dH + off;
                if (st == RS_FALLBACK) C.flags |= PERRK_FLAG_FALLBACK;
                C.state = RS_DONE;
            } else {
                relax_update(C, S, rp);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        CaseState &C = cs[c];
        if (C.state != RS_DONE) {  // unreachable with the bound above; keep gamma = 1
            C.gamma_acc = 1.0;
            C.flags |= PERRK_FLAG_FALLBACK;
            C.state = RS_DONE;
        }
        C.t += C.gamma_acc * C.dt;
        C.offset += C.H_delta;
        C.ghist[2] = C.ghist[1];
        C.ghist[1] = C.ghist[0];
        C.ghist[0] = C.gamma_acc - 1.0;
        C.gamma_prev = C.gamma_acc;
    }
}

// U <- U + gamma dt d, two doubles per thread; skipped entirely after an error.
template <int DIM>
__global__ void __launch_bounds__(256)
final_update_kernel(double *U, const double *d, const ElemInfo *elem, const CaseState *cs,
                    const int32_t *err, int64_t nelem)
{
    constexpr int NPE = Geo<DIM>::NPE, V = Geo<DIM>::V;
    if (*err != 0) return;
    const int64_t n2 = (int64_t)V * nelem * NPE / 2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t idx = 2 * i;
        const int64_t e = (idx / NPE) % nelem;
        const CaseState &C = cs[elem[e].case_id];
        const double f = C.gamma_acc * C.dt;
        double2 uu = reinterpret_cast<double2 *>(U)[i];
        const double2 dd = reinterpret_cast<const double2 *>(d)[i];
        uu.x = uu.x + f * dd.x;
        uu.y = uu.y + f * dd.y;
        reinterpret_cast<double2 *>(U)[i] = uu;
    }
}

template <int DIM>
__global__ void __launch_bounds__(256)
entropy_elem_kernel(const double *U, const ElemInfo *elem, double *partial, int64_t nelem, double gam,
                    int32_t *err)
{
    constexpr int NPE = Geo<DIM>::NPE, V = Geo<DIM>::V, EPW = Geo<DIM>::EPW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t e0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * EPW + lane / NPE;
    const bool valid = e0 < nelem;
    const int64_t e = valid ? e0 : nelem - 1;
    const int node = lane % NPE;
    double u[V];
#pragma unroll
    for (int v = 0; v < V; ++v) u[v] = U[((size_t)v * nelem + e) * NPE + node];
    double s = node_weight<DIM>(node) * entropy_density<DIM>(u, gam);
#pragma unroll
    for (int off = NPE / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (valid && node == 0) partial[e] = elem[e].jac * s;
    if (valid && !isfinite(s) && node == 0) atomicOr(err, 2);
}

__global__ void __launch_bounds__(PERRK_RED_THREADS)
case_sum_kernel(const double *partial, const int64_t *case_off, double *out)
{
    const int c = blockIdx.x;
    double o[1];
    case_sum<1>(partial, 1, case_off[c], case_off[c + 1], o);
    if (threadIdx.x == 0) out[c] = o[0];
}

__global__ void set_dt_kernel(CaseState *cs, const double *dt, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) cs[i].dt = dt[i];
}

__global__ void clear_err_kernel(int32_t *err) { *err = 0; }

__global__ void init_cases_kernel(CaseState *cs, int n)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    CaseState C = {};
    C.gamma_prev = 1.0;
    C.gamma_acc = 1.0;
    C.gamma = 1.0;
    C.state = RS_DONE;
    cs[c] = C;
}

template <int DIM, typename T, typename KT, int FLUX, int KIND>
hipError_t launch_stage_t(const StageArgs &a, const double *coef, LaunchCfg cfg, hipStream_t s)
{
    constexpr int NPE = Geo<DIM>::NPE, EPW = Geo<DIM>::EPW, NQ = Geo<DIM>::NQ;
    const int wpb = cfg.epb_mult;
    const int epb = wpb * EPW;
    if (a.n_active <= 0) return hipSuccess;
    const int blocks = (a.n_active + epb - 1) / epb;
    const size_t lds = (size_t)epb * NQ * NPE * sizeof(T);
    hipLaunchKernelGGL((stage_kernel<DIM, T, KT, FLUX, KIND>), dim3(blocks), dim3(64 * wpb), lds, s, a,
                       coef);
    return hipGetLastError();
}

template <int DIM, typename T, typename KT, int FLUX>
hipError_t launch_stage_k(int kind, const StageArgs &a, const double *coef, LaunchCfg cfg, hipStream_t s)
{
    if (kind == SK_FIRST) return launch_stage_t<DIM, T, KT, FLUX, SK_FIRST>(a, coef, cfg, s);
    if (kind == SK_MID) return launch_stage_t<DIM, T, KT, FLUX, SK_MID>(a, coef, cfg, s);
    return launch_stage_t<DIM, T, KT, FLUX, SK_LAST>(a, coef, cfg, s);
}

template <int DIM>
hipError_t launch_stage_d(int mixed, int flux, int kind, const StageArgs &a, const double *coef,
                          LaunchCfg cfg, hipStream_t s)
{
    if (mixed) {
        if (flux) return launch_stage_k<DIM, float, float, 1>(kind, a, coef, cfg, s);
        return launch_stage_k<DIM, float, float, 0>(kind, a, coef, cfg, s);
    }
    if (flux) return launch_stage_k<DIM, double, double, 1>(kind, a, coef, cfg, s);
    return launch_stage_k<DIM, double, double, 0>(kind, a, coef, cfg, s);
}

}  // namespace

hipError_t launch_stage(int dim, int mixed, int flux, int kind, const StageArgs &a, const double *coef,
                        LaunchCfg cfg, hipStream_t s)
{
    if (dim == 2) return launch_stage_d<2>(mixed, flux, kind, a, coef, cfg, s);
    return launch_stage_d<3>(mixed, flux, kind, a, coef, cfg, s);
}

hipError_t launch_relax_prepare(CaseState *cs, const int64_t *case_off, int n_cases, const double *ep,
                                int64_t nelem, RelaxParams rp, const float *mlp, hipStream_t s)
{
    hipLaunchKernelGGL(relax_prepare_kernel, dim3(n_cases), dim3(PERRK_RED_THREADS), 0, s, cs, case_off,
                       ep, nelem, rp, mlp);
    return hipGetLastError();
}

hipError_t launch_relax_pass(int dim, const double *U, const double *d, const ElemInfo *elem,
                             const CaseState *cs, double *partial, int64_t nelem, double gam,
                             hipStream_t s)
{
    const int epw = dim == 2 ? 4 : 1;
    const int64_t waves = (nelem + epw - 1) / epw;
    const int64_t blocks = (waves + 3) / 4;
    if (dim == 2)
        hipLaunchKernelGGL(relax_pass_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, U, d, elem, cs,
                           partial, nelem, gam);
    else
        hipLaunchKernelGGL(relax_pass_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, s, U, d, elem, cs,
                           partial, nelem, gam);
    return hipGetLastError();
}

hipError_t launch_relax_finalize(CaseState *cs, const int64_t *case_off, int n_cases, const double *partial,
                                 RelaxParams rp, hipStream_t s)
{
    hipLaunchKernelGGL(relax_finalize_kernel, dim3(n_cases), dim3(PERRK_RED_THREADS), 0, s, cs, case_off,
                       partial, rp);
    return hipGetLastError();
}

hipError_t launch_relax_complete(int dim, const double *U, const double *d, const ElemInfo *elem,
                                 CaseState *cs, const int64_t *case_off, int n_cases, double *partial,
                                 int64_t nelem, double gam, RelaxParams rp, hipStream_t s)
{
    if (dim == 2)
        hipLaunchKernelGGL(relax_complete_kernel<2>, dim3(n_cases), dim3(PERRK_RED_THREADS), 0, s, U, d,
                           elem, cs, case_off, partial, nelem, gam, rp);
    else
        hipLaunchKernelGGL(relax_complete_kernel<3>, dim3(n_cases), dim3(PERRK_RED_THREADS), 0, s, U, d,
                           elem, cs, case_off, partial, nelem, gam, rp);
    return hipGetLastError();
}

hipError_t launch_final_update(int dim, double *U, const double *d, const ElemInfo *elem,
                               const CaseState *cs, const int32_t *err, int64_t nelem, hipStream_t s)
{
    const int npe = dim == 2 ? 16 : 64;
    const int64_t n2 = (int64_t)(dim + 2) * nelem * npe / 2;
    int64_t blocks = (n2 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (dim == 2)
        hipLaunchKernelGGL(final_update_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, U, d, elem, cs,
                           err, nelem);
    else
        hipLaunchKernelGGL(final_update_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, s, U, d, elem, cs,
                           err, nelem);
    return hipGetLastError();
}

hipError_t launch_entropy(int dim, const double *U, const ElemInfo *elem, double *partial, double *H_out,
                          const int64_t *case_off, int n_cases, int64_t nelem, double gam, int32_t *err,
                          hipStream_t s)
{
    const int epw = dim == 2 ? 4 : 1;
    const int64_t blocks = ((nelem + epw - 1) / epw + 3) / 4;
    if (dim == 2)
        hipLaunchKernelGGL(entropy_elem_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, U, elem, partial,
                           nelem, gam, err);
    else
        hipLaunchKernelGGL(entropy_elem_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, s, U, elem, partial,
                           nelem, gam, err);
    hipLaunchKernelGGL(case_sum_kernel, dim3(n_cases), dim3(PERRK_RED_THREADS), 0, s, partial, case_off,
                       H_out);
    return hipGetLastError();
}

hipError_t launch_init_cases(CaseState *cs, int n_cases, hipStream_t s)
{
    hipLaunchKernelGGL(init_cases_kernel, dim3((n_cases + 63) / 64), dim3(64), 0, s, cs, n_cases);
    return hipGetLastError();
}

hipError_t launch_set_dt(CaseState *cs, const double *dt, int n_cases, hipStream_t s)
{
    hipLaunchKernelGGL(set_dt_kernel, dim3((n_cases + 63) / 64), dim3(64), 0, s, cs, dt, n_cases);
    return hipGetLastError();
}

hipError_t launch_clear_err(int32_t *err, hipStream_t s)
{
    hipLaunchKernelGGL(clear_err_kernel, dim3(1), dim3(1), 0, s, err);
    return hipGetLastError();
}
