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
// Each stage launches over its own list of active elements (natural order).
//
// Relaxation (Sec. 3.1): a residual pass reads U_n and d once per node and
// reduces J q [s(u + gamma dt d) - s(u)] (cancellation-free form),
// J q w(u + gamma dt d) . dt d and, when a bracket is being opened, the
// difference at a second point; one workgroup per case then sums the
// per-element partials in a fixed order and advances a Newton / bisection
// state machine held in device memory.  Per-element partials make every sum
// independent of the launch shape, so results are bitwise reproducible.

#include "perrk_internal.h"
#include "perrk_log.h"

#include <math.h>

#include <type_traits>

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

// a_t for t in 0..3, by selection (no indexed memory access)
template <typename T>
__device__ __forceinline__ T sel4(int t, T a0, T a1, T a2, T a3)
{
    const T lo = (t & 1) ? a1 : a0, hi = (t & 1) ? a3 : a2;
    return (t & 2) ? hi : lo;
}

// Dsplit[t][(t + j) & 3] for j = 1, 2, 3 (t = position of the node on its line).
template <typename T, int J>
__device__ __forceinline__ T dsplit_j(int t)
{
    if (J == 1) return sel4<T>(t, (T)(5.0 * PHI), (T)SQ5, (T)PHI, (T)-1.0);
    if (J == 2) return sel4<T>(t, (T)(-5.0 * (PHI - 1.0)), (T)(-(PHI - 1.0)), (T)(PHI - 1.0), (T)(5.0 * (PHI - 1.0)));
    return sel4<T>(t, (T)1.0, (T)(-PHI), (T)(-SQ5), (T)(-5.0 * PHI));
}

// Dsplit[t][(t + j) & 3] / 2: the weights of the Euler stage kernels' gather,
// whose two-point fluxes come doubled (halving is exact).
template <typename T, int J>
__device__ __forceinline__ T dsplit_half_j(int t)
{
    if (J == 1) return sel4<T>(t, (T)(2.5 * PHI), (T)(0.5 * SQ5), (T)(0.5 * PHI), (T)-0.5);
    if (J == 2)
        return sel4<T>(t, (T)(-2.5 * (PHI - 1.0)), (T)(-0.5 * (PHI - 1.0)), (T)(0.5 * (PHI - 1.0)),
                       (T)(2.5 * (PHI - 1.0)));
    return sel4<T>(t, (T)0.5, (T)(-0.5 * PHI), (T)(-0.5 * SQ5), (T)(-2.5 * PHI));
}

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
// L(a, b) = (a - b) / (log a - log b).  With s = a + b, z = (a - b)/s, u = z^2:
// log(a/b) = 2 z (1 + u/3 + u^2/5 + ...) = 2 z F(u), so L = (s/2) / F(u) and
// 1/L = (2/s) F(u).  Near a = b both are evaluated by series with a single
// reciprocal (1/F(u) = 1 - u/3 - 4u^2/45 - 44u^3/945 - 428u^4/14175 - ...,
// coefficients of the reciprocal power series): in double precision for
// u < 2.5e-3, truncated after u^6; in single precision for u < 1e-2, truncated
// after u^3 (the omitted terms are below the rounding unit).  Otherwise from
// log1p((a-b)/b) (flog1p in double precision, the hardware logarithm of the
// ratio in single), with reciprocals instead of divisions.
#define C_R1 (-1.0 / 3.0)
#define C_R2 (-4.0 / 45.0)
#define C_R3 (-44.0 / 945.0)
#define C_R4 (-428.0 / 14175.0)
#define C_R5 (-10196.0 / 467775.0)
#define C_R6 (-10719068.0 / 638512875.0)

// 1/x as every kernel computes it: the hardware reciprocal in single precision,
// the refined one below in double (the same expression wherever a value must
// agree bit for bit, e.g. rho / p on both sides of a face).
template <typename T>
__device__ __forceinline__ T recip(T x);
template <>
__device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// 1/x for finite nonzero x: the hardware reciprocal estimate refined by two
// Newton steps r <- r + r (1 - x r) (error within an ulp, cheaper than the
// correctly rounded division).
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

template <>
__device__ __forceinline__ double recip<double>(double x) { return rcp64(x); }

// Double-precision logarithms of the entropy arithmetic (perrk_log.h: range
// reduction to [sqrt(1/2), sqrt(2)) and the atanh series; a few ulp).
struct Rcp64 {
    __device__ double operator()(double x) const { return rcp64(x); }
};
__device__ __forceinline__ double flog(double x) { return perrk_log::log_f64(x, Rcp64{}); }
__device__ __forceinline__ double flog1p(double x) { return perrk_log::log1p_f64(x, Rcp64{}); }

// The flux arithmetic below fixes every fused multiply-add explicitly (no
// contraction left to the compiler), so that the same two-point flux gives the
// same bits whatever the code around it: a direction known at compile time or
// chosen per lane, states taken from LDS or from registers.

__device__ __forceinline__ double lmean(double a, double b)
{
#pragma clang fp contract(off)
    const double d = a - b, s = a + b;
    const double rs = rcp64(s);
    const double z = d * rs, u = z * z;
    if (u < 2.5e-3) {
        double P = fma(u, C_R6, C_R5);
        P = fma(u, P, C_R4);
        P = fma(u, P, C_R3);
        P = fma(u, P, C_R2);
        P = fma(u, P, C_R1);
        P = fma(u, P, 1.0);
        return 0.5 * s * P;
    }
    return d * rcp64(flog1p(d * rcp64(b)));
}

__device__ __forceinline__ double inv_lmean(double a, double b)
{
#pragma clang fp contract(off)
    const double d = a - b, s = a + b;
    const double rs = rcp64(s);
    const double z = d * rs, u = z * z;
    if (u < 2.5e-3) {
        double F = fma(u, 1.0 / 13.0, 1.0 / 11.0);
        F = fma(u, F, 1.0 / 9.0);
        F = fma(u, F, 1.0 / 7.0);
        F = fma(u, F, 1.0 / 5.0);
        F = fma(u, F, 1.0 / 3.0);
        F = fma(u, F, 1.0);
        return 2.0 * rs * F;
    }
    return flog1p(d * rcp64(b)) * rcp64(d);
}

__device__ __forceinline__ float lmean(float a, float b)
{
#pragma clang fp contract(off)
    const float d = a - b, s = a + b;
    const float rs = __builtin_amdgcn_rcpf(s);
    const float z = d * rs, u = z * z;
    if (u < 1.0e-2f) {
        float P = fmaf(u, (float)(0.5 * C_R3), (float)(0.5 * C_R2));
        P = fmaf(u, P, (float)(0.5 * C_R1));
        P = fmaf(u, P, 0.5f);
        return s * P;
    }
    return d * __builtin_amdgcn_rcpf(__logf(a * __builtin_amdgcn_rcpf(b)));
}

__device__ __forceinline__ float inv_lmean(float a, float b)
{
#pragma clang fp contract(off)
    const float d = a - b, s = a + b;
    const float rs = __builtin_amdgcn_rcpf(s);
    const float z = d * rs, u = z * z;
    if (u < 1.0e-2f) {
        float F = fmaf(u, (float)(2.0 / 7.0), (float)(2.0 / 5.0));
        F = fmaf(u, F, (float)(2.0 / 3.0));
        F = fmaf(u, F, 2.0f);
        return rs * F;
    }
    return __logf(a * __builtin_amdgcn_rcpf(b)) * __builtin_amdgcn_rcpf(d);
}



// ---------------------------------------------------------------- node data
template <typename T, int DIM>
struct Prim {
    T rho, v[DIM], p, beta;  // beta = rho / p
};

// Primitive variables of a double-precision state (gm1 = gamma - 1).  Sets
// bit 1 of bad for rho <= 0 or p <= 0, bit 2 for non-finite input.
template <int DIM>
__device__ __forceinline__ void make_prim_f32(const double *u, double gm1, Prim<float, DIM> &P, int &bad);

template <typename T, int DIM>
__device__ __forceinline__ void make_prim(const double *u, double gm1, Prim<T, DIM> &P, int &bad)
{
#pragma clang fp contract(off)
    if constexpr (sizeof(T) == 4) {
        make_prim_f32<DIM>(u, gm1, P, bad);
        return;
    }
    const double rho = u[0];
    const double ir = rcp64(rho);
    double v[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) v[k] = u[1 + k] * ir;
    double ke = u[1] * v[0];
#pragma unroll
    for (int k = 1; k < DIM; ++k) ke = fma(u[1 + k], v[k], ke);
    const double p = gm1 * fma(-0.5, ke, u[DIM + 1]);
    double sum = u[0];
#pragma unroll
    for (int k = 1; k < DIM + 2; ++k) sum += u[k];
    if (!isfinite(sum)) bad |= 2;  // a sum of finite values can overflow only beyond 1e308
    else if (!(rho > 0.0) || !(p > 0.0)) bad |= 1;
    P.rho = (T)rho;
#pragma unroll
    for (int k = 0; k < DIM; ++k) P.v[k] = (T)v[k];
    P.p = (T)p;
    P.beta = (T)(rho * recip<double>(p));
}

// Single-precision variant from a single-precision state (reciprocals by the
// hardware instruction).  A state whose components exceed the single-precision
// range counts as non-finite.
template <int DIM>
__device__ __forceinline__ void prim_f32(const float *uf, double gm1, Prim<float, DIM> &P, int &bad)
{
#pragma clang fp contract(off)
    float sum = uf[0];
#pragma unroll
    for (int k = 1; k < DIM + 2; ++k) sum += uf[k];
    const float rho = uf[0];
    const float ir = __builtin_amdgcn_rcpf(rho);
#pragma unroll
    for (int k = 0; k < DIM; ++k) P.v[k] = uf[1 + k] * ir;
    float ke = uf[1] * P.v[0];
#pragma unroll
    for (int k = 1; k < DIM; ++k) ke = fmaf(uf[1 + k], P.v[k], ke);
    const float p = (float)gm1 * fmaf(-0.5f, ke, uf[DIM + 1]);
    if (!isfinite(sum)) bad |= 2;
    else if (!(rho > 0.0f) || !(p > 0.0f)) bad |= 1;
    P.rho = rho;
    P.p = p;
    P.beta = rho * recip<float>(p);
}

// From a double-precision state, rounded to single precision first.
template <int DIM>
__device__ __forceinline__ void make_prim_f32(const double *u, double gm1, Prim<float, DIM> &P, int &bad)
{
    float uf[DIM + 2];
#pragma unroll
    for (int k = 0; k < DIM + 2; ++k) uf[k] = (float)u[k];
    prim_f32<DIM>(uf, gm1, P, bad);
}

// Velocity component d of a state with a runtime d, by selection of values.
template <typename T, int DIM>
__device__ __forceinline__ T vdir(const Prim<T, DIM> &P, int d)
{
    if (DIM == 2) return d == 0 ? P.v[0] : P.v[1];
    return d == 0 ? P.v[0] : (d == 1 ? P.v[1] : P.v[DIM - 1]);
}

// Ranocha's entropy-conservative, kinetic-energy-preserving two-point flux in
// direction d (runtime): f_rho = {rho}_log {v_d}, f_m = f_rho {v} + {p} e_d,
// f_E = f_rho (v_L.v_R / 2 + 1 / ((gamma-1) {rho/p}_log)) + (p_L v_R,d + p_R v_L,d) / 2.
//
// TWICE: returns 2 f, which saves the halvings of the means (every scaling by 2
// is exact, so 2 f has the bits of f times two).
template <typename T, int DIM, bool TWICE = false>
__device__ __forceinline__ void flux_ec(int d, const Prim<T, DIM> &L, const Prim<T, DIM> &R, T inv_gm1, T *f)
{
#pragma clang fp contract(off)
    const T rm = lmean(L.rho, R.rho);
    const T ibm = inv_lmean(L.beta, R.beta);
    if constexpr (TWICE) {
        T sv[DIM];  // sums of the velocity components: twice their means
#pragma unroll
        for (int k = 0; k < DIM; ++k) sv[k] = L.v[k] + R.v[k];
        const T vl = vdir<T, DIM>(L, d), vr = vdir<T, DIM>(R, d);
        const T svd = DIM == 2 ? (d == 0 ? sv[0] : sv[1]) : (d == 0 ? sv[0] : (d == 1 ? sv[1] : sv[DIM - 1]));
        const T fr2 = rm * svd;     // 2 f_rho
        const T fr = (T)0.5 * fr2;  // f_rho
        const T sp = L.p + R.p;     // twice the mean pressure
        T vv = L.v[0] * R.v[0];
#pragma unroll
        for (int k = 1; k < DIM; ++k) vv = fma(L.v[k], R.v[k], vv);
        f[0] = fr2;
#pragma unroll
        for (int k = 0; k < DIM; ++k) f[1 + k] = fma(fr, sv[k], k == d ? sp : (T)0);
        f[DIM + 1] = fma(fr2, fma((T)0.5, vv, inv_gm1 * ibm), fma(L.p, vr, R.p * vl));
        return;
    }
    T va[DIM];  // arithmetic means of the velocity components
#pragma unroll
    for (int k = 0; k < DIM; ++k) va[k] = (T)0.5 * (L.v[k] + R.v[k]);
    const T vl = vdir<T, DIM>(L, d), vr = vdir<T, DIM>(R, d);
    const T vm = DIM == 2 ? (d == 0 ? va[0] : va[1]) : (d == 0 ? va[0] : (d == 1 ? va[1] : va[DIM - 1]));
    const T fr = rm * vm;
    const T pa = (T)0.5 * (L.p + R.p);
    T vv = L.v[0] * R.v[0];
#pragma unroll
    for (int k = 1; k < DIM; ++k) vv = fma(L.v[k], R.v[k], vv);
    f[0] = fr;
#pragma unroll
    for (int k = 0; k < DIM; ++k) f[1 + k] = fma(fr, va[k], k == d ? pa : (T)0);
    f[DIM + 1] = fma(fr, fma((T)0.5, vv, inv_gm1 * ibm), (T)0.5 * fma(L.p, vr, R.p * vl));
}

// Dissipative surface fluxes in direction d, selected at run time (the value is
// uniform over the launch):
//   PERRK_FLUX_HLL   two-wave HLL with Davis speeds min/max(v_n -+ c)
//   PERRK_FLUX_LLF   local Lax-Friedrichs: HLL with speeds -+max(|v_n| + c)
//   PERRK_FLUX_HLLE  HLL with Einfeldt speeds: the Davis outer speeds widened by
//                    the Roe-averaged (sqrt(rho)-weighted) v_n -+ c
//   PERRK_FLUX_HLLC  three waves (Toro): Davis outer speeds, contact speed s*,
//                    star state of the side of the contact that holds x = 0
// The conserved states are rebuilt from the primitive ones.
template <typename T, int DIM>
__device__ __forceinline__ void flux_diss(int kind, int d, const Prim<T, DIM> &L, const Prim<T, DIM> &R, T gam,
                                          T inv_gm1, T *f)
{
    const T vl = vdir<T, DIM>(L, d), vr = vdir<T, DIM>(R, d);
    const T cl = sqrt(gam * L.p / L.rho), cr = sqrt(gam * R.p / R.rho);
    T lmin = fmin(vl - cl, vr - cr);
    T lmax = fmax(vl + cl, vr + cr);
    T uL[DIM + 2], uR[DIM + 2], fl[DIM + 2], fr[DIM + 2];
    T kl = 0, kr = 0;
    uL[0] = L.rho;
    uR[0] = R.rho;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        uL[1 + k] = L.rho * L.v[k];
        uR[1 + k] = R.rho * R.v[k];
        kl += uL[1 + k] * L.v[k];
        kr += uR[1 + k] * R.v[k];
    }
    uL[DIM + 1] = L.p * inv_gm1 + (T)0.5 * kl;
    uR[DIM + 1] = R.p * inv_gm1 + (T)0.5 * kr;
#pragma unroll
    for (int k = 0; k < DIM + 1; ++k) {
        fl[k] = uL[k] * vl;
        fr[k] = uR[k] * vr;
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        if (k == d) {
            fl[1 + k] += L.p;
            fr[1 + k] += R.p;
        }
    }
    fl[DIM + 1] = (uL[DIM + 1] + L.p) * vl;
    fr[DIM + 1] = (uR[DIM + 1] + R.p) * vr;
    if (kind == PERRK_FLUX_LLF) {
        lmax = fmax(fabs(vl) + cl, fabs(vr) + cr);
        lmin = -lmax;
    } else if (kind == PERRK_FLUX_HLLE) {
        const T sl = sqrt(L.rho), sr = sqrt(R.rho);
        const T iw = (T)1 / (sl + sr);
        T v2 = 0, vn = 0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const T vt = (sl * L.v[k] + sr * R.v[k]) * iw;
            v2 += vt * vt;
            vn = k == d ? vt : vn;
        }
        const T ht = (sl * (uL[DIM + 1] + L.p) / L.rho + sr * (uR[DIM + 1] + R.p) / R.rho) * iw;
        const T ct = sqrt((gam - (T)1) * (ht - (T)0.5 * v2));
        lmin = fmin(vl - cl, vn - ct);
        lmax = fmax(vr + cr, vn + ct);
    }
    if (lmin >= (T)0) {
#pragma unroll
        for (int k = 0; k < DIM + 2; ++k) f[k] = fl[k];
    } else if (lmax <= (T)0) {
#pragma unroll
        for (int k = 0; k < DIM + 2; ++k) f[k] = fr[k];
    } else if (kind == PERRK_FLUX_HLLC) {
        const T ml = L.rho * (lmin - vl), mr = R.rho * (lmax - vr);
        const T ss = (R.p - L.p + ml * vl - mr * vr) / (ml - mr);
        const bool left = ss >= (T)0;
        const T sk = left ? lmin : lmax, mk = left ? ml : mr, vk = left ? vl : vr;
        const T rk = left ? L.rho : R.rho, pk = left ? L.p : R.p;
        const T fac = mk / (sk - ss);
        T us[DIM + 2];
        us[0] = fac;
#pragma unroll
        for (int k = 0; k < DIM; ++k) us[1 + k] = fac * (k == d ? ss : (left ? L.v[k] : R.v[k]));
        const T ek = left ? uL[DIM + 1] : uR[DIM + 1];
        us[DIM + 1] = fac * (ek / rk + (ss - vk) * (ss + pk / mk));
#pragma unroll
        for (int k = 0; k < DIM + 2; ++k) f[k] = (left ? fl[k] : fr[k]) + sk * (us[k] - (left ? uL[k] : uR[k]));
    } else {
        const T inv = (T)1 / (lmax - lmin);
#pragma unroll
        for (int k = 0; k < DIM + 2; ++k)
            f[k] = (lmax * fl[k] - lmin * fr[k] + lmin * lmax * (uR[k] - uL[k])) * inv;
    }
}

// Entropy variables of s = -rho log(p rho^-gamma):
// w = (gamma - log(p rho^-gamma) - (gamma-1) rho |v|^2 / (2p), (gamma-1) rho v / p, -(gamma-1) rho / p).
// (Reciprocals by rcp64: the stage epilogues form these per node, and correctly
// rounded divisions would cost about as much as one logarithm.)
template <int DIM>
__device__ __forceinline__ void entropy_vars(const double *u, double gam, double *w)
{
#pragma clang fp contract(off)
    const double rho = u[0];
    const double ir = rcp64(rho);
    double m2 = u[1] * u[1];
#pragma unroll
    for (int k = 1; k < DIM; ++k) m2 = fma(u[1 + k], u[1 + k], m2);
    const double p = (gam - 1.0) * fma(-0.5 * m2, ir, u[DIM + 1]);
    const double rp = rho * rcp64(p);
    const double g1rp = (gam - 1.0) * rp;
    w[0] = fma(-0.5 * g1rp * m2, ir * ir, gam - fma(-gam, flog(rho), flog(p)));
#pragma unroll
    for (int k = 0; k < DIM; ++k) w[1 + k] = g1rp * u[1 + k] * ir;
    w[DIM + 1] = -g1rp;
}

// s(u) = -rho (log p - gamma log rho).
template <int DIM>
__device__ __forceinline__ double entropy_density(const double *u, double gam)
{
#pragma clang fp contract(off)
    double m2 = u[1] * u[1];
#pragma unroll
    for (int k = 1; k < DIM; ++k) m2 = fma(u[1 + k], u[1 + k], m2);
    const double p = (gam - 1.0) * (u[DIM + 1] - 0.5 * m2 / u[0]);
    return -u[0] * fma(-gam, flog(u[0]), flog(p));
}

// log1p(x): series x - x^2/2 + ... + x^9/9 for |x| < 1e-2 (omitted term < 1e-20/10),
// flog1p otherwise.  The relaxation arithmetic below fixes its fused
// multiply-adds (no contraction left to the compiler), so that an evaluation
// gives the same bits in every kernel that makes it (the last stage, the
// launched passes, the completion kernel), whatever code surrounds it.
__device__ __forceinline__ double log1p_small(double x)
{
#pragma clang fp contract(off)
    if (fabs(x) < 1.0e-2) {
        double P = fma(x, 1.0 / 9.0, -1.0 / 8.0);
        P = fma(x, P, 1.0 / 7.0);
        P = fma(x, P, -1.0 / 6.0);
        P = fma(x, P, 1.0 / 5.0);
        P = fma(x, P, -1.0 / 4.0);
        P = fma(x, P, 1.0 / 3.0);
        P = fma(x, P, -1.0 / 2.0);
        P = fma(x, P, 1.0);
        return x * P;
    }
    return flog1p(x);
}

// At one node, with du = g dt d: the entropy difference s(u + du) - s(u)
// (cancellation-free form) and w(u + du) . (dt d), sharing the intermediate
// quantities.  With rho' = rho + drho, p' = p + dp:
//   s' - s = -drho log(p' rho'^-gamma) - rho [log1p(dp/p) - gamma log1p(drho/rho)],
//   log(p' rho'^-gamma) = log(p rho^-gamma) + log1p(dp/p) - gamma log1p(drho/rho),
//   w' = (gamma - log(p' rho'^-gamma) - (gamma-1) |m'|^2 / (2 rho' p'), (gamma-1) m'/p', -(gamma-1) rho'/p').
template <int DIM>
__device__ __forceinline__ void relax_node(const double *u, const double *dv, double g, double dt, double gam,
                                           double &ds, double &wd)
{
#pragma clang fp contract(off)
    const double rho = u[0];
    const double gdt = g * dt;
    double du[DIM + 2];
#pragma unroll
    for (int v = 0; v < DIM + 2; ++v) du[v] = gdt * dv[v];
    const double drho = du[0], rho1 = rho + drho;
    // reciprocals by rcp64 (within an ulp; a correctly rounded division costs
    // about three times as many instructions, and this runs per node and pass)
    const double ir = rcp64(rho), ir1 = rcp64(rho1);
    double mdm = u[1] * du[1], dm2 = du[1] * du[1], m2 = u[1] * u[1];
#pragma unroll
    for (int k = 1; k < DIM; ++k) {
        mdm = fma(u[1 + k], du[1 + k], mdm);
        dm2 = fma(du[1 + k], du[1 + k], dm2);
        m2 = fma(u[1 + k], u[1 + k], m2);
    }
    const double g1 = gam - 1.0;
    // p = (gamma-1) (E - |m|^2 / (2 rho)),
    // dp = (gamma-1) (dE - (m.dm + |dm|^2/2) / rho' + drho |m|^2 / (2 rho rho'))
    const double p = g1 * fma(-0.5 * m2, ir, u[DIM + 1]);
    const double dp = g1 * fma(0.5 * drho * m2, ir * ir1, fma(-fma(0.5, dm2, mdm), ir1, du[DIM + 1]));
    const double p1 = p + dp;
    const double lp = log1p_small(dp * rcp64(p)), lr = log1p_small(drho * ir);
    const double lpr = fma(-gam, lr, lp);                 // log1p(dp/p) - gamma log1p(drho/rho)
    const double sth1 = fma(-gam, flog(rho), flog(p)) + lpr;  // log(p' rho'^-gamma)
    ds = fma(-drho, sth1, -rho * lpr);
    const double ip1 = rcp64(p1), gip = g1 * ip1;
    const double m12 = fma(2.0, mdm, m2) + dm2;  // |m'|^2
    double dot = fma(-0.5 * g1 * m12, ir1 * ip1, gam - sth1) * dv[0];
#pragma unroll
    for (int k = 0; k < DIM; ++k) dot = fma(gip * (u[1 + k] + du[1 + k]), dv[1 + k], dot);
    dot = fma(-gip * rho1, dv[DIM + 1], dot);
    wd = dt * dot;
}


// Raw data of one node for its stage state: U_n, K_1 and K_{i-1}.  Every load
// depends only on the element index, so a lane issues all of them at once;
// double-precision stages read K_{i-1} even where its coefficient is zero (it
// may then hold stale values, which the combination discards by selection,
// never by multiplication), single-precision stages skip it there.
// Single-precision stages after the first read U_n from its single-precision
// copy (UT = float): they round U_n to single precision anyway, so the copy
// gives the same bits with half the bytes.
template <int V, typename KT, typename UT = double>
struct NodeRaw {
    UT u[V];
    KT k1[V], kp[V];
};

// Node arrays are read and written with buffer instructions: one resource per
// field (base = array + v * field, range = the field's bytes; scalar registers)
// and one 32-bit byte offset per lane, shared by every field and array of the
// same element size, so an access costs no vector address arithmetic.  The
// node count of all cases stays below 2^29 (PERRK_MAX_NODES), so an FP64 field
// spans less than 4 GiB and every lane offset fits 32 bits.
typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef unsigned int u32x2 __attribute__((__vector_size__(8)));
constexpr int RSRC_WORD3 = 0x00020000;  // word 3 of a raw gfx9 buffer resource: 32-bit data format

template <typename T>
__device__ __forceinline__ Rsrc field_rsrc(const void *base, int v, size_t field)
{
    T *p = const_cast<T *>(static_cast<const T *>(base)) + (size_t)v * field;
    return __builtin_amdgcn_make_buffer_rsrc(p, 0, (int)perrk_buffer_range(field, sizeof(T)), RSRC_WORD3);
}

template <typename T>
__device__ __forceinline__ T bload(Rsrc r, uint32_t o)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)o, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)o, 0, 0));
}

template <typename T>
__device__ __forceinline__ void bstore(T x, Rsrc r, uint32_t o)
{
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, (int)o, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, (int)o, 0, 0);
}

// base[i] with a 32-bit byte offset (tables indexed by element, case or level
// are far below 4 GiB).
template <typename T>
__device__ __forceinline__ const T &elt(const T *base, uint32_t i)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + i * (uint32_t)sizeof(T));
}

// kp_on = false skips the K_{i-1} loads (their coefficient is zero: the first
// stage a level evaluates after the first).
template <int DIM, typename KT, int KIND, typename UT>
__device__ __forceinline__ void load_raw(const StageArgs &a, int e, int node, NodeRaw<Geo<DIM>::V, KT, UT> &r,
                                         bool kp_on = true)
{
    constexpr int NPE = Geo<DIM>::NPE, V = Geo<DIM>::V;
    const size_t field = (size_t)a.nelem * NPE;
    const uint32_t n = (uint32_t)e * NPE + node;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        if constexpr (sizeof(UT) == 4) r.u[v] = bload<float>(field_rsrc<float>(a.U32, v, field), n * 4u);
        else r.u[v] = bload<double>(field_rsrc<double>(a.U, v, field), n * 8u);
        if (KIND != SK_FIRST) {
            r.k1[v] = bload<KT>(field_rsrc<KT>(a.K1, v, field), n * (uint32_t)sizeof(KT));
            r.kp[v] = kp_on ? bload<KT>(field_rsrc<KT>(a.Kp, v, field), n * (uint32_t)sizeof(KT)) : (KT)0;
        }
    }
}

// U_{n,i} = U_n + dt (c1 K_1 + cp K_{i-1}) with the node's level coefficients.
// This, the primitive variables and the entropy variables fix their fused
// multiply-adds explicitly (contraction off): a lane forms its own state and,
// for its face node, the neighbour's from the neighbour's data, and the two
// must have the bits the neighbour's own lanes give them (both sides of a face
// then form the same flux).
template <int V, typename KT, int KIND>
__device__ __forceinline__ void combine(const NodeRaw<V, KT> &r, double dt, double c1, double cp, double *u)
{
#pragma clang fp contract(off)
#pragma unroll
    for (int v = 0; v < V; ++v) {
        double x = r.u[v];
        if (KIND != SK_FIRST) {
            double s = c1 * (double)r.k1[v];
            s = (cp != 0.0) ? fma(cp, (double)r.kp[v], s) : s;
            x = fma(dt, s, x);
        }
        u[v] = x;
    }
}

// The same in single precision (stages whose fluxes are single precision): U_n is
// rounded first, the combination is formed in single precision.
template <int V, typename KT, int KIND, typename UT>
__device__ __forceinline__ void combine_f32(const NodeRaw<V, KT, UT> &r, double dt, float c1, float cp, float *u)
{
#pragma clang fp contract(off)
    const float fdt = (float)dt, fc1 = c1, fcp = cp;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        float x = (float)r.u[v];
        if (KIND != SK_FIRST) {
            float s = fc1 * (float)r.k1[v];
            s = (cp != 0.0f) ? fmaf(fcp, (float)r.kp[v], s) : s;
            x = fmaf(fdt, s, x);
        }
        u[v] = x;
    }
}

// Synchronisation of the stage kernel's LDS phases.  Each wavefront reads and
// writes only its own element slots, and the LDS operations of one wavefront
// are performed in issue order, so no workgroup barrier is needed: the
// wavefront-scope fences and the wave barrier only keep the compiler from
// moving LDS accesses across the phase boundary.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroups are handed to the 8 XCDs of the device round-robin; renumber them
// so that each XCD works on one contiguous range of logical blocks (neighbouring
// elements then share that XCD's L2).
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// ---------------------------------------------------------------- per-element values
// Every lane of an element slot needs the same per-element values: the active
// entry, dt of the element's case, the level coefficients of the element and of
// its face neighbours, the element's metric.  A few lanes load them and the
// others take them by cross-lane reads: a load by every lane would move each
// value through the vector memory path once per lane, and those repeated bytes
// were close to half of the path's traffic in the stage kernels.

// Lanes 2k and 2k + 1 load the two 16-byte halves of the active entry of the
// wavefront's slot k (list index li0 + k, clamped to the list); other lanes
// return zeros.
template <int EPW>
__device__ __forceinline__ int4 wave_entry_part(const void *active, int li0, int n_active, int lane)
{
    int4 r = make_int4(0, 0, 0, 0);
    if (lane < 2 * EPW) {
        const int j = min(li0 + (lane >> 1), n_active - 1);
        r = elt(reinterpret_cast<const int4 *>(active), 2u * (uint32_t)j + (uint32_t)(lane & 1));
    }
    return r;
}

__device__ __forceinline__ int4 shfl4(const int4 &v, int src)
{
    return make_int4(__shfl(v.x, src), __shfl(v.y, src), __shfl(v.z, src), __shfl(v.w, src));
}

// Lanes 0 .. 2 PERRK_MAXR - 1 hold the stage's coefficient table (c_1 of level r
// at lane r, c_p at lane PERRK_MAXR + r); coef_of reads entry j of it.
__device__ __forceinline__ double wave_coef_table(const double *coef, int lane)
{
    return lane < 2 * PERRK_MAXR ? elt(coef, (uint32_t)lane) : 0.0;
}

// Lane k < EPW loads dt of slot k's case and the metric and Jacobian of slot k's
// element (entry halves in `part`); the slot's lanes take them with slot_value.
template <int DIM, int EPW>
struct SlotVals {
    double dt, h[DIM], jac;
};

template <int DIM, int EPW, bool DT>
__device__ __forceinline__ SlotVals<DIM, EPW> wave_slot_vals(const StageArgs &a, const int4 &part, int lane)
{
    const int src = 2 * (lane % EPW);
    const uint32_t ex = (uint32_t)__shfl(part.x, src) & PERRK_NBR_MASK;
    const uint32_t cy = (uint32_t)__shfl(part.y, src);
    SlotVals<DIM, EPW> r;
    r.dt = 0.0;
    r.jac = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) r.h[d] = 0.0;
    if (lane < EPW) {
        const ElemInfo &ek = elt(a.elem, ex);
#pragma unroll
        for (int d = 0; d < DIM; ++d) r.h[d] = ek.metric[d];
        r.jac = ek.jac;
        if (DT) r.dt = elt(a.cs, cy).dt;
    }
    return r;
}

// The values of slot es, for every lane of the slot; the metric and Jacobian in
// an ElemInfo (its other fields are not used by the stage kernels).
template <int DIM, int EPW>
__device__ __forceinline__ void slot_value(const SlotVals<DIM, EPW> &v, int es, double &dt, ElemInfo &ei)
{
    dt = __shfl(v.dt, es);
#pragma unroll
    for (int d = 0; d < 3; ++d) ei.metric[d] = d < DIM ? __shfl(v.h[d < DIM ? d : 0], es) : 0.0;
    ei.jac = __shfl(v.jac, es);
}

// ---------------------------------------------------------------- stage kernel
// LDS per element slot (flux precision T):
//   prim[NPE][NQ]   own stage state per node: rho, v_0..v_{DIM-1}, p
//   sf[V][NFN]      lifted surface flux of each face node (+-6 f*), NFN = 2 DIM NPE/4
//   vf[V][NPP]      two-point fluxes of the pairs of the current phase (up to two directions)
template <int DIM>
struct SG {
    static constexpr int NPE = Geo<DIM>::NPE, V = DIM + 2, EPW = Geo<DIM>::EPW;
    static constexpr int NLINE = NPE / 4;        // LGL lines per direction
    static constexpr int NFN = 2 * DIM * NLINE;  // face nodes
    static constexpr int NPD = 6 * NLINE;        // node pairs per direction
    static constexpr int NPP = 2 * NPD;          // pairs held per phase
    static constexpr int NQ = DIM + 2;
};

// Element slot in LDS, in words of T: primitives [node][NQ], then rho/p per
// node where stored (BETA), the lifted surface fluxes sf[V][NFN] and the pair
// fluxes vf[V][VS].  Single-precision slots and the one-direction slots of
// quadrilaterals store rho/p once per node, which saves a quarter-rate
// reciprocal per read; the other double-precision slots recompute it where they
// read a node (their smaller slots keep more waves resident: a hexahedron's
// one-direction slot already fills the LDS at four waves per SIMD).  VS: pair
// fluxes of one phase, NPP (two directions) or, where the directions are done
// one at a time (SPLIT), NPD.
template <int DIM, typename T, bool SPLIT = false>
struct SL {
    static constexpr bool BETA = sizeof(T) == 4 || (SPLIT && DIM == 2);
    static constexpr int PRIM = SG<DIM>::NQ * SG<DIM>::NPE + (BETA ? SG<DIM>::NPE : 0);
    static constexpr int VS = SPLIT ? SG<DIM>::NPD : SG<DIM>::NPP;
    static constexpr int SLOT = PRIM + SG<DIM>::V * (SG<DIM>::NFN + VS);  // LDS words per slot
};

// Stages with the EC fluxes can take the directions one at a time (pairs and
// faces of x, then of y; hexahedra z, x, y: the same fluxes and sums in the same
// order), which halves the pair-flux area of a slot; the autotuner chooses per
// stage.
template <int DIM, int FLUX, bool ONE_DIR>
struct SplitDirs {
    static constexpr bool ON = ONE_DIR && FLUX == 0;
};

// Node of line l (the other coordinates) at position t along direction d.
template <int DIM>
__device__ __forceinline__ int line_node(int d, int l, int t)
{
    if (DIM == 2) return d == 0 ? t + 4 * l : l + 4 * t;
    if (d == 0) return t + 4 * (l & 3) + 16 * (l >> 2);
    if (d == 1) return (l & 3) + 4 * t + 16 * (l >> 2);
    return l + 16 * t;
}

// Line index of a node in direction d (also its position on the faces normal to d).
template <int DIM>
__device__ __forceinline__ int node_line(int d, int node)
{
    const int i = node & 3, j = (node >> 2) & 3, k = node >> 4;
    if (DIM == 2) return d == 0 ? j : i;
    if (d == 0) return j + 4 * k;
    if (d == 1) return i + 4 * k;
    return i + 4 * j;
}

__device__ __forceinline__ int node_pos(int d, int node)
{
    return d == 0 ? (node & 3) : (d == 1 ? ((node >> 2) & 3) : (node >> 4));
}

// Pairs of positions on a line, k = 0..5: (0,1),(0,2),(0,3),(1,2),(1,3),(2,3).
__device__ __forceinline__ void pair_pos(int k, int &a, int &b)
{
    a = k < 3 ? 0 : (k < 5 ? 1 : 2);
    b = k < 3 ? k + 1 : (k < 5 ? k - 1 : 3);
}

// Pair index k of positions (t, (t + j) & 3), j = 1, 2, 3.
template <int J>
__device__ __forceinline__ int pair_k(int t)
{
    if (J == 1) return sel4<int>(t, 0, 3, 5, 2);
    if (J == 2) return sel4<int>(t, 1, 4, 1, 4);
    return sel4<int>(t, 2, 0, 3, 5);
}

// Face nodes of a wavefront: EPW * NFN of them (64 in 2D, 96 in 3D), spread over
// the lanes in FR rounds; face node g = lane + 64 r belongs to element slot
// g / NFN, which is the lane's own slot (2D: 16 face nodes per quadrilateral;
// 3D: one element per wavefront).
template <int DIM>
struct FaceRounds {
    static constexpr int N = (SG<DIM>::EPW * SG<DIM>::NFN + 63) / 64;
};

template <int DIM>
struct FaceNode {
    int q, d, side, own;  // face-node slot, direction, side (1 = +), own node on the face
};

template <int DIM>
__device__ __forceinline__ bool face_node(int r, int lane, FaceNode<DIM> &F, int &nn)
{
    constexpr int EPW = SG<DIM>::EPW, NFN = SG<DIM>::NFN, NLINE = SG<DIM>::NLINE;
    const int g = lane + 64 * r;
    const int es = g / NFN;
    F.q = g - es * NFN;
    const int f = F.q / NLINE, l = F.q - f * NLINE;
    F.d = f >> 1;
    F.side = f & 1;
    F.own = line_node<DIM>(F.d, l, F.side ? 3 : 0);
    nn = line_node<DIM>(F.d, l, F.side ? 0 : 3);  // matching node of the neighbour
    return g < EPW * NFN;
}

// Lane -> node pair of round rd over the directions [D0, D0 + ND): element slot
// es, direction offset dd, line l, pair k.  Bit fields of the lane index:
//   2D (ND = 2): 4 slots x 2 directions x 4 lines x 2 pairs per round
//                (lane = 16 es + 8 dd + 2 l + k - 2 rd), 3 rounds;
//   3D, ND = 2:  2 directions x 16 lines x 2 pairs per round (lane = 32 dd + 2 l +
//                k - 2 rd), 3 rounds; with UNI, round 0 holds pairs k = 0..3 of every
//                line in direction D0 (lane = 4 l + k), round 2 the same in direction
//                D0 + 1 and round 1 the pairs k = 4, 5 of both (lane = 32 dd + 2 l +
//                k - 4), so that two of the three rounds form their fluxes in a
//                direction fixed at compile time;
//   3D, ND = 1:  round 0: lane = 4 l + k; round 1: pairs k = 4, 5 on lanes 0..31
//                (2 l + k - 4), with UNI on lanes 32..63, leaving lanes 0..31 to the
//                surface fluxes of the faces normal to D0 merged into that round.
template <int DIM, int ND>
struct PairRounds {
    static_assert(DIM == 3 || ND == 2, "2D evaluates both directions in one phase");
    static constexpr int N = (DIM == 3 && ND == 1) ? 2 : 3;
};

template <int DIM, int ND, bool UNI = false>
__device__ __forceinline__ bool pair_of(int rd, int lane, int &es, int &dd, int &l, int &k)
{
    if (DIM == 3 && ND == 1) {
        es = 0;
        dd = 0;
        if (rd == 0) {
            l = lane >> 2;
            k = lane & 3;
            return true;
        }
        l = (lane >> 1) & 15;
        k = 4 + (lane & 1);
        return UNI ? lane >= 32 : lane < 32;
    }
    if (DIM == 2) {
        es = lane >> 4;
        dd = (lane >> 3) & 1;
        l = (lane >> 1) & 3;
        k = 2 * rd + (lane & 1);
        return true;
    }
    es = 0;
    if (!UNI) {
        dd = lane >> 5;
        l = (lane >> 1) & 15;
        k = 2 * rd + (lane & 1);
        return true;
    }
    if (rd != 1) {
        dd = rd == 0 ? 0 : 1;
        l = lane >> 2;
        k = lane & 3;
        return true;
    }
    dd = lane >> 5;
    l = (lane >> 1) & 15;
    k = 4 + (lane & 1);
    return true;
}

// Primitive variables of a node in LDS: rho, v_0..v_{DIM-1}, p, contiguous per
// node (one or two wide LDS reads); rho/p stored beside them (slots with BETA),
// or formed on reading with the same expression make_prim uses (so that both
// sides of a face, and both kinds of slot, see the same bits).
template <typename T, int DIM, bool SPLIT = false>
__device__ __forceinline__ void lds_put_prim(T *slot, int node, const Prim<T, DIM> &P)
{
    constexpr int NQ = SG<DIM>::NQ, NPE = SG<DIM>::NPE;
    T *q = slot + node * NQ;
    q[0] = P.rho;
#pragma unroll
    for (int k = 0; k < DIM; ++k) q[1 + k] = P.v[k];
    q[DIM + 1] = P.p;
    if constexpr (SL<DIM, T, SPLIT>::BETA) slot[NQ * NPE + node] = P.beta;
}

template <typename T, int DIM, bool SPLIT = false>
__device__ __forceinline__ void lds_get_prim(const T *slot, int node, Prim<T, DIM> &P)
{
    constexpr int NQ = SG<DIM>::NQ, NPE = SG<DIM>::NPE;
    const T *q = slot + node * NQ;
    P.rho = q[0];
#pragma unroll
    for (int k = 0; k < DIM; ++k) P.v[k] = q[1 + k];
    P.p = q[DIM + 1];
    if constexpr (SL<DIM, T, SPLIT>::BETA) P.beta = slot[NQ * NPE + node];
    else P.beta = P.rho * recip<T>(P.p);
}

// Central two-point flux (f(u_A) + f(u_B)) / 2 in direction d.  In the split
// form sum_m Dsplit[t][m] f#(t, m) it gives D f - B f / q (the rows of D sum to
// zero), which with the lifted surface flux is the strong form and, by the SBP
// property q D + D^T q = B, exactly the standard weak form.
// TWICE: returns 2 f (the same sums without the final halving).
template <typename T, int DIM, bool TWICE = false>
__device__ __forceinline__ void flux_central(int d, const Prim<T, DIM> &A, const Prim<T, DIM> &B, T inv_gm1, T *f)
{
#pragma clang fp contract(off)
    const T va = vdir<T, DIM>(A, d), vb = vdir<T, DIM>(B, d);
    T ka = A.v[0] * A.v[0], kb = B.v[0] * B.v[0];
#pragma unroll
    for (int k = 1; k < DIM; ++k) {
        ka = fma(A.v[k], A.v[k], ka);
        kb = fma(B.v[k], B.v[k], kb);
    }
    const T h = TWICE ? (T)1 : (T)0.5;
    const T ma = A.rho * va, mb = B.rho * vb;
    f[0] = h * (ma + mb);
#pragma unroll
    for (int k = 0; k < DIM; ++k) f[1 + k] = h * (fma(ma, A.v[k], mb * B.v[k]) + (k == d ? A.p + B.p : (T)0));
    const T ea = fma(A.p, inv_gm1, (T)0.5 * A.rho * ka), eb = fma(B.p, inv_gm1, (T)0.5 * B.rho * kb);
    f[DIM + 1] = h * fma(ea + A.p, va, (eb + B.p) * vb);
}

// Field-by-field choice between two node states (values, so that both stay in
// registers).
template <typename T, int DIM>
__device__ __forceinline__ Prim<T, DIM> pick(bool c, const Prim<T, DIM> &X, const Prim<T, DIM> &Y)
{
    Prim<T, DIM> P;
    P.rho = c ? X.rho : Y.rho;
#pragma unroll
    for (int k = 0; k < DIM; ++k) P.v[k] = c ? X.v[k] : Y.v[k];
    P.p = c ? X.p : Y.p;
    P.beta = c ? X.beta : Y.beta;
    return P;
}

// Two-point volume fluxes of the pairs of directions [D0, D0 + ND), one pair per
// lane and round, written to vf of the pair's element slot: the EC flux, or the
// central flux for the weak form.  FACES (3D, ND = 1, EC surface flux): the free
// lanes 0..31 of round 1 form the surface fluxes of face nodes 64..95, the faces
// normal to D0, from the own face node in LDS and the neighbour's state PNF, and
// write them lifted to sf, as the surface-flux rounds do for the other faces.
// UNI: the pair mapping with rounds of one direction (used with FACES, whose
// lanes it leaves free, and by the hexahedra's other phase in the same kernels).
template <int DIM, typename T, int D0, int ND, bool WEAK, bool FACES = false, bool UNI = FACES>
__device__ __forceinline__ void volume_pairs(T *lds, int wave, int lane, T inv_gm1,
                                             const FaceNode<DIM> *FF = nullptr, const Prim<T, DIM> *PNF = nullptr,
                                             bool fvf = false)
{
    static_assert(!FACES || (DIM == 3 && ND == 1 && !WEAK), "faces merge into the one-direction 3D phase");
    constexpr int EPW = SG<DIM>::EPW, NPD = SG<DIM>::NPD, NPP = SG<DIM>::NPP, V = SG<DIM>::V;
    constexpr int SLOT = SL<DIM, T>::SLOT, PRIM = SL<DIM, T>::PRIM, NFN = SG<DIM>::NFN;
    constexpr int NR = PairRounds<DIM, ND>::N;
    // every round's two nodes are read before the first flux is formed (the
    // pair-flux writes below may not be moved above these reads), so that one
    // LDS latency is exposed instead of one per round and the rounds' flux
    // arithmetic is independent
    Prim<T, DIM> A[NR], B[NR];
    int pv[NR];
    bool ok[NR];
    T *vfs[NR];
    const bool face_lane = FACES && lane < 32;
#pragma unroll
    for (int rd = 0; rd < NR; ++rd) {
        int es, dd, l, k;
        ok[rd] = pair_of<DIM, ND, UNI>(rd, lane, es, dd, l, k);
        int ta, tb;
        pair_pos(k, ta, tb);
        const int d = D0 + dd;
        T *slot = lds + (size_t)(wave * EPW + es) * SLOT;
        if (FACES && rd == 1) {
            // pair lanes read both nodes, face lanes their own face node; the face
            // lanes' minus / plus states are then the own node and the neighbour in
            // the order of the face's side
            Prim<T, DIM> X, Y;
            lds_get_prim<T, DIM>(slot, face_lane ? FF->own : line_node<DIM>(d, l, ta), X);
            lds_get_prim<T, DIM>(slot, line_node<DIM>(d, l, tb), Y);  // (a node of the slot on every lane)
            Y = pick<T, DIM>(face_lane, *PNF, Y);
            const bool swap = face_lane && FF->side == 0;
            A[rd] = pick<T, DIM>(swap, Y, X);
            B[rd] = pick<T, DIM>(swap, X, Y);
            ok[rd] = face_lane ? fvf : ok[rd];
        } else if (ok[rd]) {
            lds_get_prim<T, DIM>(slot, line_node<DIM>(d, l, ta), A[rd]);
            lds_get_prim<T, DIM>(slot, line_node<DIM>(d, l, tb), B[rd]);
        }
        vfs[rd] = slot + PRIM + V * NFN;
        pv[rd] = dd * NPD + l * 6 + k;
    }
#pragma unroll
    for (int rd = 0; rd < NR; ++rd) {
        if (!ok[rd]) continue;
        int es, dd, l, k;
        pair_of<DIM, ND, UNI>(rd, lane, es, dd, l, k);
        const int d = D0 + dd;
        T f[V];
        if (WEAK) flux_central<T, DIM, true>(d, A[rd], B[rd], inv_gm1, f);
        else flux_ec<T, DIM, true>(d, A[rd], B[rd], inv_gm1, f);
        if (FACES && rd == 1 && face_lane) {
            const T lift = FF->side ? (T)3 : (T)-3;  // (the flux is doubled)
            T *sf = vfs[rd] - V * NFN;
#pragma unroll
            for (int v = 0; v < V; ++v) sf[v * NFN + FF->q] = lift * f[v];
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) vfs[rd][v * NPP + pv[rd]] = f[v];
        }
    }
}

// One direction D at a time (SPLIT slots): the direction's pairs and the face
// nodes of the faces normal to it in two rounds, all with the EC flux in
// direction D.
//   round 0: pairs k = 0..3 (2D: lane = 16 es + 4 l + k; 3D: lane = 4 l + k);
//   round 1: the lanes whose face node (F, the neighbour's state PN) lies on a
//            face normal to D form that face's flux from the own node in LDS and
//            PN; the other lanes take pairs k = 4, 5 (2D: es = lane / 16,
//            l = (lane / 2) mod 4; 3D: l = (lane / 2) mod 16).  2D face node of a
//            lane: q = lane mod 16, x faces for q < 8; 3D: x faces on lanes 0..31
//            and y faces on lanes 32..63 of the first face round, z faces on
//            lanes 0..31 of the second.
// Pair fluxes go to vf (NPD per variable), face fluxes lifted to sf, exactly as
// the two-direction rounds and the surface-flux round store them.  The rounds
// run one after the other (fewer registers held than reading both first).
template <int DIM, typename T, int D>
__device__ __forceinline__ void pairs_and_faces(T *lds, int wave, int lane, T inv_gm1, const FaceNode<DIM> &F,
                                                const Prim<T, DIM> &PN)
{
    constexpr int EPW = SG<DIM>::EPW, NPD = SG<DIM>::NPD, V = SG<DIM>::V, NFN = SG<DIM>::NFN;
    constexpr int SLOT = SL<DIM, T, true>::SLOT, PRIM = SL<DIM, T, true>::PRIM;
    const int es = DIM == 2 ? lane >> 4 : 0;
    T *slot = lds + (size_t)(wave * EPW + es) * SLOT;
    T *sf = slot + PRIM;
    T *vf = sf + V * NFN;
    const bool face_lane = DIM == 2 ? ((lane >> 3) & 1) == D : (D == 1 ? lane >= 32 : lane < 32);
    T f[V];
    {
        const int l = DIM == 2 ? (lane >> 2) & 3 : lane >> 2, k = lane & 3;
        int ta, tb;
        pair_pos(k, ta, tb);
        Prim<T, DIM> A, B;
        lds_get_prim<T, DIM, true>(slot, line_node<DIM>(D, l, ta), A);
        lds_get_prim<T, DIM, true>(slot, line_node<DIM>(D, l, tb), B);
        flux_ec<T, DIM, true>(D, A, B, inv_gm1, f);
#pragma unroll
        for (int v = 0; v < V; ++v) vf[v * NPD + l * 6 + k] = f[v];
    }
    const int l = DIM == 2 ? (lane >> 1) & 3 : (lane >> 1) & 15, k = 4 + (lane & 1);
    int ta, tb;
    pair_pos(k, ta, tb);
    Prim<T, DIM> X, Y;
    lds_get_prim<T, DIM, true>(slot, face_lane ? F.own : line_node<DIM>(D, l, ta), X);
    lds_get_prim<T, DIM, true>(slot, line_node<DIM>(D, l, tb), Y);  // (a node of the slot on every lane)
    Y = pick<T, DIM>(face_lane, PN, Y);
    const bool swap = face_lane && F.side == 0;
    flux_ec<T, DIM, true>(D, pick<T, DIM>(swap, Y, X), pick<T, DIM>(swap, X, Y), inv_gm1, f);
    if (face_lane) {
        const T lift = F.side ? (T)3 : (T)-3;  // (the flux is doubled)
#pragma unroll
        for (int v = 0; v < V; ++v) sf[v * NFN + F.q] = lift * f[v];
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) vf[v * NPD + l * 6 + k] = f[v];
    }
}

// Gather table of the single-precision stages, one copy per wavefront in LDS
// (16 words; lanes 0-15 copy it from here at the start): for each position t on
// a line, Dsplit[t][(t + j) & 3] / 2 for j = 1, 2, 3 in single precision and the
// three pair indices pair_k<j>(t) in 4-bit fields.  Each lane reads its row with
// one LDS load per direction instead of forming six values by selection.
constexpr uint32_t gtab_word(int i)
{
    const int t = i >> 2, j = i & 3;
    if (j == 3) {
        const int k1[4] = {0, 3, 5, 2}, k2[4] = {1, 4, 1, 4}, k3[4] = {2, 0, 3, 5};
        return (uint32_t)(k1[t] | (k2[t] << 4) | (k3[t] << 8));
    }
    const float w[3][4] = {{(float)(2.5 * PHI), (float)(0.5 * SQ5), (float)(0.5 * PHI), (float)-0.5},
                           {(float)(-2.5 * (PHI - 1.0)), (float)(-0.5 * (PHI - 1.0)), (float)(0.5 * (PHI - 1.0)),
                            (float)(2.5 * (PHI - 1.0))},
                           {(float)0.5, (float)(-0.5 * PHI), (float)(-0.5 * SQ5), (float)(-2.5 * PHI)}};
    return __builtin_bit_cast(uint32_t, w[j][t]);
}
__device__ const uint32_t GATHER_TAB[16] = {
    gtab_word(0), gtab_word(1), gtab_word(2),  gtab_word(3),  gtab_word(4),  gtab_word(5),  gtab_word(6),  gtab_word(7),
    gtab_word(8), gtab_word(9), gtab_word(10), gtab_word(11), gtab_word(12), gtab_word(13), gtab_word(14), gtab_word(15)};
constexpr int GTAB_WORDS = 16;

// Adds -(2/h_d) [sum_{m != t} Dsplit[t][m] f#(t, m) + lifted surface flux] of the
// directions [d0, d0 + nd) to du (node lane); hn[d] = -(2/h_d) in flux precision;
// tab: the wavefront's gather table (single precision only).  The pair fluxes
// are stored doubled, 2 f#, and weighted by Dsplit / 2 (the same products).
template <int DIM, typename T, int D0, int ND, int VS = SG<DIM>::NPP>
__device__ __forceinline__ void gather(const T *slot, int node, const T *hn, const T *tab, T *du)
{
#pragma clang fp contract(off)
    constexpr int d0 = D0, nd = ND;
    constexpr int NPD = SG<DIM>::NPD, NPP = VS, V = SG<DIM>::V, PRIM = SL<DIM, T, VS == NPD>::PRIM;
    constexpr int NFN = SG<DIM>::NFN, NLINE = SG<DIM>::NLINE;
    const T *sf = slot + PRIM;
    const T *vf = sf + V * NFN;
#pragma unroll
    for (int dd = 0; dd < nd; ++dd) {
        const int d = d0 + dd;
        const int t = node_pos(d, node);
        const int l = node_line<DIM>(d, node);
        T acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0;
        const int pb = dd * NPD + l * 6;
        int p1, p2, p3;
        T w1, w2, w3;
        if constexpr (sizeof(T) == 4) {
            const float4 row = *reinterpret_cast<const float4 *>(tab + 4 * t);
            const uint32_t pk = __builtin_bit_cast(uint32_t, row.w);
            w1 = row.x;
            w2 = row.y;
            w3 = row.z;
            p1 = pb + (int)(pk & 15u);
            p2 = pb + (int)((pk >> 4) & 15u);
            p3 = pb + (int)(pk >> 8);
        } else {
            p1 = pb + pair_k<1>(t);
            p2 = pb + pair_k<2>(t);
            p3 = pb + pair_k<3>(t);
            w1 = dsplit_half_j<T, 1>(t);
            w2 = dsplit_half_j<T, 2>(t);
            w3 = dsplit_half_j<T, 3>(t);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            acc[v] = fma(w1, vf[v * NPP + p1], acc[v]);
            acc[v] = fma(w2, vf[v * NPP + p2], acc[v]);
            acc[v] = fma(w3, vf[v * NPP + p3], acc[v]);
        }
        if (t == 0 || t == 3) {
            const int q = (2 * d + (t == 3 ? 1 : 0)) * NLINE + l;
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] += sf[v * NFN + q];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) du[v] = fma(hn[d], acc[v], du[v]);
    }
}


}  // namespace

namespace {

// T: flux arithmetic; KT: stage storage.  Lane = node of the element slot
// lane / NPE of its wavefront.  Memory access is arranged so that the global
// loads of a lane form at most three dependent levels, all issued before the
// first LDS phase boundary: the active entry (element, level, case); then the
// element's own U_n / K_1 / K_{i-1}, dt, its level coefficients and the
// neighbour words of its face nodes; then the neighbours' data at the matching
// nodes.  A wavefront never waits for the other wavefronts of its workgroup.
template <int DIM, typename T, typename KT, int FLUX, int KIND, bool ONE_DIR>
__global__ void __launch_bounds__(64 * PERRK_MAX_WPB) stage_kernel(const StageArgs a, const double *coef)
{
    constexpr bool SPLIT = SplitDirs<DIM, FLUX, ONE_DIR>::ON;
    constexpr int NPE = SG<DIM>::NPE, V = SG<DIM>::V, EPW = SG<DIM>::EPW, SLOT = SL<DIM, T, SPLIT>::SLOT;
    constexpr int PRIM = SL<DIM, T, SPLIT>::PRIM, NFN = SG<DIM>::NFN, FR = FaceRounds<DIM>::N;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int es = lane / NPE;
    const int eslot = wave * EPW + es;
    const int node = lane % NPE;
    const int epb = (int)(blockDim.x >> 6) * EPW;
    const int li0 = xcd_block(blockIdx.x, gridDim.x) * epb + wave * EPW;  // the wavefront's first entry
    const bool valid = li0 + es < a.n_active;
    // Single-precision stages (bound by memory latency as much as by arithmetic) load the active
    // entries {element | level, case, nbr 0, nbr 1}, {nbr 2 .. nbr 5}, the
    // coefficient table, dt and the metric with a few lanes and broadcast them,
    // and take a neighbour in the workgroup from LDS; double-precision stages
    // (bound by their arithmetic, where the broadcasts and the second path
    // would lengthen each wavefront) load them per lane.
    constexpr bool WL = sizeof(T) == 4;
    constexpr bool LOCAL = WL && DIM == 2;
    const int4 part = WL ? wave_entry_part<EPW>(a.active, li0, a.n_active, lane) : make_int4(0, 0, 0, 0);
    // level coefficients: single precision in single-precision stages (the precision
    // their stage states are formed in), shuffled from the lanes that loaded them
    using CT = typename std::conditional<WL, float, double>::type;
    const CT cf = (WL && KIND != SK_FIRST) ? (CT)wave_coef_table(coef, lane) : (CT)0;
    int4 act, act2;
    if constexpr (WL) {
        act = shfl4(part, 2 * es);
        act2 = shfl4(part, 2 * es + 1);
    } else {
        const int4 *ap = reinterpret_cast<const int4 *>(a.active);
        const uint32_t ai = (uint32_t)(valid ? li0 + es : a.n_active - 1);
        act = elt(ap, 2u * ai);
        act2 = elt(ap, 2u * ai + 1u);
    }
    const int e = (int)((uint32_t)act.x & PERRK_NBR_MASK);
    const int lvl = (int)((uint32_t)act.x >> PERRK_NBR_SHIFT);
    T *slot = lds + (size_t)eslot * SLOT;
    const T inv_gm1 = (T)a.inv_gm1;
    int bad = 0;
    // single precision: the wavefront's gather table after the workgroup's element slots
    T *gtab = WL ? lds + (size_t)epb * SLOT + wave * GTAB_WORDS : nullptr;
    const uint32_t gword = (WL && lane < GTAB_WORDS) ? elt(GATHER_TAB, (uint32_t)lane) : 0u;

    // ---- loads
    SlotVals<DIM, EPW> sv{};
    if constexpr (WL) sv = wave_slot_vals<DIM, EPW, KIND != SK_FIRST>(a, part, lane);
    CT c1 = 0, cp = 0;
    if (KIND != SK_FIRST) {
        c1 = WL ? __shfl(cf, lvl) : (CT)elt(coef, (uint32_t)lvl);
        cp = WL ? __shfl(cf, PERRK_MAXR + lvl) : (CT)elt(coef, (uint32_t)(PERRK_MAXR + lvl));
    }
    // single-precision middle stages read the single-precision copy of U_n (the last
    // stage reads U_n in double precision: the first residual evaluation needs it)
    using UT = typename std::conditional<sizeof(T) == 4 && KIND == SK_MID, float, double>::type;
    NodeRaw<V, KT, UT> own;
    // single-precision stages have their level coefficients at hand already (from
    // cross-lane reads) and skip K_{i-1} where its coefficient is zero
    load_raw<DIM, KT, KIND>(a, e, node, own, !WL || cp != (CT)0);
    FaceNode<DIM> F[FR];
    bool fv[FR];
    NodeRaw<V, KT, UT> nr[FR];
    CT nc1[FR], ncp[FR];
    int nnr[FR], lk[FR];  // the neighbour's node; its element slot in this workgroup, else -1
#pragma unroll
    for (int r = 0; r < FR; ++r) {
        fv[r] = face_node<DIM>(r, lane, F[r], nnr[r]);
        const int f = 2 * F[r].d + F[r].side;
        const uint32_t w = (uint32_t)(f < 2 ? (f == 0 ? act.z : act.w)
                                            : sel4<int>(f - 2, act2.x, act2.y, act2.z, act2.w));
        const int nb = (int)(w & PERRK_NBR_MASK);
        lk[r] = -1;
        if constexpr (LOCAL) {
            // 2D lists record the neighbour's list position relative to the entry's
            const int code = (int)(((uint32_t)act2.w >> (6 * f)) & 63u);
            const int t = eslot + code - 31;
            if (code != 63 && t >= 0 && t < epb) lk[r] = t;
        }
        // (cross-lane reads with every lane active: a lane that is switched off
        // does not provide its value)
        nc1[r] = 0;
        ncp[r] = 0;
        if (KIND != SK_FIRST) {
            const int lv = (int)(w >> PERRK_NBR_SHIFT);
            nc1[r] = WL ? __shfl(cf, lv) : (CT)elt(coef, (uint32_t)lv);
            ncp[r] = WL ? __shfl(cf, PERRK_MAXR + lv) : (CT)elt(coef, (uint32_t)(PERRK_MAXR + lv));
        }
        if (lk[r] < 0) load_raw<DIM, KT, KIND>(a, nb, nnr[r], nr[r], !WL || ncp[r] != (CT)0);
    }
    double dt = 0.0;
    ElemInfo ei;
    if constexpr (WL) {
        slot_value<DIM, EPW>(sv, es, dt, ei);
    } else {
        if (KIND != SK_FIRST) dt = elt(a.cs, (uint32_t)act.y).dt;
        const ElemInfo &eg = elt(a.elem, (uint32_t)e);
#pragma unroll
        for (int d = 0; d < 3; ++d) ei.metric[d] = d < DIM ? eg.metric[d] : 0.0;
        ei.jac = eg.jac;
    }

    // ---- own stage state, published in LDS; neighbour states (same case, hence
    // the same dt) kept in registers.  Single-precision stages form the states in
    // single precision, the others in double.
    double u[V];
    Prim<T, DIM> PN[FR];
    {
        Prim<T, DIM> me;
        if constexpr (sizeof(T) == 4) {
            float uf[V];
            combine_f32<V, KT, KIND>(own, dt, c1, cp, uf);
            prim_f32<DIM>(uf, a.gm1, me, bad);
#pragma unroll
            for (int v = 0; v < V; ++v) u[v] = (double)uf[v];  // for the entropy production
#pragma unroll
            for (int r = 0; r < FR; ++r) {
                if (lk[r] >= 0) continue;
                float unf[V];
                combine_f32<V, KT, KIND>(nr[r], dt, nc1[r], ncp[r], unf);
                prim_f32<DIM>(unf, a.gm1, PN[r], bad);
            }
        } else {
            combine<V, KT, KIND>(own, dt, c1, cp, u);
            make_prim<T, DIM>(u, a.gm1, me, bad);
#pragma unroll
            for (int r = 0; r < FR; ++r) {
                if (lk[r] >= 0) continue;
                double un[V];
                combine<V, KT, KIND>(nr[r], dt, nc1[r], ncp[r], un);
                make_prim<T, DIM>(un, a.gm1, PN[r], bad);
            }
        }
        lds_put_prim<T, DIM, SPLIT>(slot, node, me);
        if (WL && lane < GTAB_WORDS) reinterpret_cast<uint32_t *>(gtab)[lane] = gword;
    }
    if constexpr (KIND == SK_FIRST) {
        // the single-precision copy of U_n for the later single-precision stages
        if (a.U32_out != nullptr && valid) {
            const size_t field = (size_t)a.nelem * NPE;
            const uint32_t o4 = ((uint32_t)e * NPE + node) * 4u;
#pragma unroll
            for (int v = 0; v < V; ++v) bstore<float>((float)own.u[v], field_rsrc<float>(a.U32_out, v, field), o4);
        }
    }
    if constexpr (LOCAL) {
        // every slot's state is published before any lane reads a neighbour's from
        // its slot (formed by the neighbour's own lanes with the same arithmetic);
        // slots are not written in the primitives' area after this point
        __syncthreads();
#pragma unroll
        for (int r = 0; r < FR; ++r)
            if (lk[r] >= 0) lds_get_prim<T, DIM>(lds + (size_t)lk[r] * SLOT, nnr[r], PN[r]);
    } else {
        wave_lds_sync();
    }

    // ---- surface fluxes, lifted: +6 f* on right faces, -6 f* on left (+-1/q_boundary).
    // Hexahedra with the EC surface flux form those of the faces normal to direction
    // 2 (face nodes 64..95, the second round) in the half-empty last round of that
    // direction's pairs instead.
    // Quadrilaterals with the EC surface flux form all their face fluxes in the
    // rounds of the direction-by-direction phases below.
    constexpr bool MERGE = DIM == 3 && FLUX == 0;
#pragma unroll
    for (int r = 0; r < FR; ++r) {
        if (SPLIT || (MERGE && r == 1)) continue;
        if (!fv[r]) continue;
        Prim<T, DIM> PO;
        lds_get_prim<T, DIM>(slot, F[r].own, PO);
        const bool sd = F[r].side != 0;
        // minus / plus states of the face, selected field by field (values, not
        // addresses, so that everything stays in registers)
        Prim<T, DIM> L, R;
        L.rho = sd ? PO.rho : PN[r].rho;
        R.rho = sd ? PN[r].rho : PO.rho;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            L.v[k] = sd ? PO.v[k] : PN[r].v[k];
            R.v[k] = sd ? PN[r].v[k] : PO.v[k];
        }
        L.p = sd ? PO.p : PN[r].p;
        R.p = sd ? PN[r].p : PO.p;
        L.beta = sd ? PO.beta : PN[r].beta;
        R.beta = sd ? PN[r].beta : PO.beta;
        T fs[V];
        T lift;  // +-6 f* (the EC flux comes doubled: +-3)
        if (FLUX && a.flux != PERRK_FLUX_EC) {
            flux_diss<T, DIM>(a.flux, F[r].d, L, R, (T)a.gam, inv_gm1, fs);
            lift = sd ? (T)6 : (T)-6;
        } else {
            flux_ec<T, DIM, true>(F[r].d, L, R, inv_gm1, fs);
            lift = sd ? (T)3 : (T)-3;
        }
        T *sf = slot + PRIM;
#pragma unroll
        for (int v = 0; v < V; ++v) sf[v * NFN + F[r].q] = lift * fs[v];
    }

    // ---- volume fluxes and the gather, which sums K_i = -(volume + surface terms)
    T hn[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) hn[d] = -(T)ei.metric[d];
    T du[V];
#pragma unroll
    for (int v = 0; v < V; ++v) du[v] = 0;
    const bool weak = FLUX && a.volume;  // uniform over the launch
    if constexpr (SPLIT && DIM == 2) {
        constexpr int NPD = SG<DIM>::NPD;
        pairs_and_faces<DIM, T, 0>(lds, wave, lane, inv_gm1, F[0], PN[0]);
        wave_lds_sync();
        gather<DIM, T, 0, 1, NPD>(slot, node, hn, gtab, du);
        wave_lds_sync();
        pairs_and_faces<DIM, T, 1>(lds, wave, lane, inv_gm1, F[0], PN[0]);
        wave_lds_sync();
        gather<DIM, T, 1, 1, NPD>(slot, node, hn, gtab, du);
    } else if constexpr (SPLIT) {
        // z first, as the merged two-phase form sums it
        constexpr int NPD = SG<DIM>::NPD;
        pairs_and_faces<DIM, T, 2>(lds, wave, lane, inv_gm1, F[FR - 1], PN[FR - 1]);
        wave_lds_sync();
        gather<DIM, T, 2, 1, NPD>(slot, node, hn, gtab, du);
        wave_lds_sync();
        pairs_and_faces<DIM, T, 0>(lds, wave, lane, inv_gm1, F[0], PN[0]);
        wave_lds_sync();
        gather<DIM, T, 0, 1, NPD>(slot, node, hn, gtab, du);
        wave_lds_sync();
        pairs_and_faces<DIM, T, 1>(lds, wave, lane, inv_gm1, F[0], PN[0]);
        wave_lds_sync();
        gather<DIM, T, 1, 1, NPD>(slot, node, hn, gtab, du);
    } else if constexpr (MERGE) {
        // direction 2 first (its pairs and the merged faces), then directions 0 and 1
        volume_pairs<DIM, T, 2, 1, false, true>(lds, wave, lane, inv_gm1, &F[1], &PN[1], fv[1]);
        wave_lds_sync();
        gather<DIM, T, 2, 1>(slot, node, hn, gtab, du);
        wave_lds_sync();
        volume_pairs<DIM, T, 0, 2, false, false, true>(lds, wave, lane, inv_gm1);
        wave_lds_sync();
        gather<DIM, T, 0, 2>(slot, node, hn, gtab, du);
    } else {
        if (weak) volume_pairs<DIM, T, 0, 2, true>(lds, wave, lane, inv_gm1);
        else volume_pairs<DIM, T, 0, 2, false>(lds, wave, lane, inv_gm1);
        wave_lds_sync();
        gather<DIM, T, 0, 2>(slot, node, hn, gtab, du);
    }
    if constexpr (DIM == 3 && !MERGE) {
        wave_lds_sync();
        if (weak) volume_pairs<DIM, T, 2, 1, true>(lds, wave, lane, inv_gm1);
        else volume_pairs<DIM, T, 2, 1, false>(lds, wave, lane, inv_gm1);
        wave_lds_sync();
        gather<DIM, T, 2, 1>(slot, node, hn, gtab, du);
    }

    // last stage: the double-precision copies of K_1 / K_{S-1} that enter d are
    // loaded after the flux work (fewer registers held through it)
    double dacc[V];  // last stage: the contributions to d accumulated by earlier stages
    if constexpr (KIND == SK_LAST) {
        const size_t field = (size_t)a.nelem * NPE;
        const uint32_t o8 = ((uint32_t)e * NPE + node) * 8u;
#pragma unroll
        for (int v = 0; v < V; ++v) dacc[v] = a.d_has ? bload<double>(field_rsrc<double>(a.d_out, v, field), o8) : 0.0;
    }
    double k64sm1[V], k64_1[V];  // (double-precision stages only; mixed precision keeps these copies)
    if constexpr (KIND == SK_LAST && sizeof(T) == 8) {
        const size_t field = (size_t)a.nelem * NPE;
        const uint32_t o8 = ((uint32_t)e * NPE + node) * 8u;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            k64sm1[v] = a.k64_sm1 ? bload<double>(field_rsrc<double>(a.k64_sm1, v, field), o8) : 0.0;
            k64_1[v] = a.k64_1 ? bload<double>(field_rsrc<double>(a.k64_1, v, field), o8) : 0.0;
        }
    }
    // K_i in double (for d, the double copy and the entropy production)
    double k[V];
#pragma unroll
    for (int v = 0; v < V; ++v) k[v] = (double)du[v];

    // last stage: the direction d = b_S K_S + b_{S-1} K_{S-1} + b_1 K_1 (+ earlier terms)
    double dvv[V];
    if constexpr (KIND == SK_LAST) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            double dv = a.bs * k[v];
            double ksm1, k1;
            if constexpr (sizeof(T) == 8 && sizeof(KT) == 4) {
                // mixed precision: the double copies, kept wherever the weight is nonzero
                // (so the single-precision K_1, K_{S-1} need not stay live through the
                // flux work: 16-20 fewer VGPRs, one more wavefront per SIMD on hexahedra)
                ksm1 = k64sm1[v];
                k1 = k64_1[v];
            } else {
                ksm1 = (double)own.kp[v];
                k1 = (double)own.k1[v];
            }
            if (a.bsm1 != 0.0) dv += a.bsm1 * ksm1;
            if (a.b1 != 0.0) dv += a.b1 * k1;
            if (a.d_has) dv += dacc[v];
            dvv[v] = dv;
        }
    }
    if (valid) {
        const size_t field = (size_t)a.nelem * NPE;
        const uint32_t n = (uint32_t)e * NPE + node, o8 = n * 8u, ok = n * (uint32_t)sizeof(KT);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (KIND == SK_LAST) {
                bstore<double>(dvv[v], field_rsrc<double>(a.d_out, v, field), o8);
            } else {
                bstore<KT>((KT)du[v], field_rsrc<KT>(a.Kout, v, field), ok);
                if (a.k64_out) bstore<double>(k[v], field_rsrc<double>(a.k64_out, v, field), o8);
                if (a.acc_mode) {
                    double dv = a.b_acc * k[v];
                    if (a.acc_mode == 2) dv += bload<double>(field_rsrc<double>(a.d_out, v, field), o8);
                    bstore<double>(dv, field_rsrc<double>(a.d_out, v, field), o8);
                }
            }
        }
    }
    if constexpr (KIND == SK_LAST) {
        // the first residual evaluation of the relaxation solve, at the case's starting
        // value gamma_0: per element J sum q [s(u_n + gamma_0 dt d) - s(u_n)],
        // J sum q w(u_n + gamma_0 dt d) . dt d and sum |d|, with the same per-node
        // arithmetic and the same butterfly as a residual pass, so the partials are
        // those a pass over the stored d would give, bit for bit
        if (a.rx_partial != nullptr) {
            const double g0 = elt(a.cs, (uint32_t)act.y).gamma;
            double un[V];
#pragma unroll
            for (int v = 0; v < V; ++v) un[v] = (double)own.u[v];
            double sabs = 0.0;
#pragma unroll
            for (int v = 0; v < V; ++v) sabs += fabs(dvv[v]);
            double ds, wd;
            relax_node<DIM>(un, dvv, g0, dt, a.gam, ds, wd);
            const double q = node_weight<DIM>(node);
            double sr = q * ds, srp = q * wd;
#pragma unroll
            for (int off = NPE / 2; off >= 1; off >>= 1) {
                sr += __shfl_xor(sr, off);
                srp += __shfl_xor(srp, off);
                sabs += __shfl_xor(sabs, off);
            }
            if (valid && node == 0) {
                double *pp = a.rx_partial + (size_t)e * 4;
                pp[0] = ei.jac * sr;
                pp[1] = ei.jac * srp;
                pp[2] = 0.0;
                pp[3] = sabs;
            }
        }
    }
    if (a.ep_partial != nullptr) {
        // entropy production with K_i as it enters d: double when a double copy is
        // kept (or K is stored in double), else as stored
        double w[V];
        entropy_vars<DIM>(u, a.gam, w);
        double dot = 0.0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const double kv = (KIND == SK_LAST || a.k64_out || sizeof(KT) == 8) ? k[v] : (double)(KT)du[v];
            dot += w[v] * kv;
        }
        double sm = node_weight<DIM>(node) * dot;
#pragma unroll
        for (int off = NPE / 2; off >= 1; off >>= 1) sm += __shfl_xor(sm, off);
        if (valid && node == 0) a.ep_partial[e] = ei.jac * sm;
    }
    if (bad && valid) atomicOr(a.err, bad);
}

// ---------------------------------------------------------------- ideal GLM-MHD
// Nine conserved variables per node, u = (rho, rho v_1..3, E, B_1..3, psi), on
// 2D meshes (all three vector components carried), double precision.  The
// system is u_t + sum_d [d_d f_d + Phi(u) d_d B_d + Phi_d(u) d_d psi] = 0 with
//   p = (gamma-1) (E - rho |v|^2/2 - |B|^2/2 - psi^2/2),
//   f_rho = rho v_d, f_m = rho v v_d + (p + |B|^2/2) e_d - B B_d,
//   f_E = v_d (rho |v|^2/2 + gamma p/(gamma-1) + |B|^2) - B_d (v.B) + c_h psi B_d,
//   f_B = v_d B - B_d v + c_h psi e_d, f_psi = c_h B_d,
//   Phi = (0, B, v.B, v, 0) (Powell), Phi_d = (0, 0, 0, 0, v_d psi, 0, 0, 0, v_d) (GLM).
// Volume term: flux differencing with an EC two-point flux, or the central flux
// (the weak form).  Surface flux: EC, local Lax-Friedrichs or central.  The
// non-conservative terms: Phi(u_i) times the split-form sum of the pair means
// {B_d} plus the lifted face means, which is the strong-form derivative of B_d
// with the face mean as interface value (and the same for psi).
constexpr int MHD_V = 9;
constexpr int MHD_NC = 11;  // flux components + the means of B_d and psi
constexpr int MHD_NQ = 9;   // primitives per node in LDS: rho, v_1..3, p, B_1..3, psi
// LDS doubles per element: the primitives, the lifted face fluxes and face means
// (MHD_NC per face node), the pair fluxes (MHD_V per pair; the gather forms the
// pair means of B_d and psi from the primitives) of both directions, or of one
// direction at a time (ONE_DIR: 584 instead of 752 doubles, 8 instead of 6
// wavefronts per compute unit).
template <bool ONE_DIR>
constexpr int mhd_slot()
{
    return MHD_NQ * 16 + MHD_NC * SG<2>::NFN + MHD_V * (ONE_DIR ? SG<2>::NPD : SG<2>::NPP);
}

struct PrimM {
    double rho, v[3], p, B[3], psi;
};

__device__ __forceinline__ void make_prim_mhd(const double *u, double gm1, PrimM &P, int &bad)
{
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < MHD_V; ++k) sum += u[k];
    const double rho = u[0];
    const double ir = rcp64(rho);
    double kin = 0.0, mag = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        P.v[k] = u[1 + k] * ir;
        kin += u[1 + k] * P.v[k];
        P.B[k] = u[5 + k];
        mag += u[5 + k] * u[5 + k];
    }
    P.psi = u[8];
    const double p = gm1 * (u[4] - 0.5 * kin - 0.5 * mag - 0.5 * u[8] * u[8]);
    if (!isfinite(sum)) bad |= 2;
    else if (!(rho > 0.0) || !(p > 0.0)) bad |= 1;
    P.rho = rho;
    P.p = p;
}

__device__ __forceinline__ void mhd_put(double *slot, int node, const PrimM &P)
{
    double *q = slot + node * MHD_NQ;
    q[0] = P.rho;
    q[1] = P.v[0];
    q[2] = P.v[1];
    q[3] = P.v[2];
    q[4] = P.p;
    q[5] = P.B[0];
    q[6] = P.B[1];
    q[7] = P.B[2];
    q[8] = P.psi;
}

__device__ __forceinline__ void mhd_get(const double *slot, int node, PrimM &P)
{
    const double *q = slot + node * MHD_NQ;
    P.rho = q[0];
    P.v[0] = q[1];
    P.v[1] = q[2];
    P.v[2] = q[3];
    P.p = q[4];
    P.B[0] = q[5];
    P.B[1] = q[6];
    P.B[2] = q[7];
    P.psi = q[8];
}

__device__ __forceinline__ double sel2(int d, double a, double b) { return d == 0 ? a : b; }

// Physical flux in direction d (0 or 1) from primitive variables.
// The GLM-MHD fluxes fix their fused multiply-adds explicitly (contraction off),
// as the Euler fluxes do: a pair flux then has the same bits whether its
// direction is a compile-time constant (one direction at a time) or a per-lane
// value (two directions per phase).
__device__ __forceinline__ double dot3(const double *a, const double *b)
{
#pragma clang fp contract(off)
    return fma(a[2], b[2], fma(a[1], b[1], a[0] * b[0]));
}

__device__ __forceinline__ void mhd_flux_phys(int d, const PrimM &P, double gam, double inv_gm1, double c_h, double *f)
{
#pragma clang fp contract(off)
    const double vn = sel2(d, P.v[0], P.v[1]), Bn = sel2(d, P.B[0], P.B[1]);
    const double vB = dot3(P.v, P.B), B2 = dot3(P.B, P.B), v2 = dot3(P.v, P.v);
    const double ptot = fma(0.5, B2, P.p);
    const double mn = P.rho * vn;
    f[0] = mn;
#pragma unroll
    for (int k = 0; k < 3; ++k) f[1 + k] = fma(mn, P.v[k], fma(-P.B[k], Bn, k == d ? ptot : 0.0));
    f[4] = fma(vn, fma(0.5 * P.rho, v2, fma(gam * inv_gm1, P.p, B2)), fma(-Bn, vB, c_h * P.psi * Bn));
#pragma unroll
    for (int k = 0; k < 3; ++k) f[5 + k] = fma(vn, P.B[k], fma(-P.v[k], Bn, k == d ? c_h * P.psi : 0.0));
    f[8] = c_h * Bn;
}

// Entropy-conservative two-point flux (with beta = rho / (2p), arithmetic means
// {.}, logarithmic means {.}_log, p~ = {rho} / (2 {beta})):
//   f_rho = {rho}_log {v_d}
//   f_m   = f_rho {v} - (B_d,A B_B + B_d,B B_A)/2 + (p~ + B_A.B_B/2) e_d
//   f_B   = {v_d B - B_d v} + c_h {psi} e_d,  f_psi = c_h {B_d}
//   f_E   = f_rho (1/(2 (gamma-1) {beta}_log) - {|v|^2}/2) + f_m.{v} + f_B.{B}
//           + f_psi {psi} - {v_d |B|^2}/2 + {B_d} {v.B} - c_h {psi B_d}
__device__ __forceinline__ void mhd_flux_ec(int d, const PrimM &A, const PrimM &B, double inv_gm1, double c_h,
                                            double *f)
{
#pragma clang fp contract(off)
    const double ba = 0.5 * A.rho * rcp64(A.p), bb = 0.5 * B.rho * rcp64(B.p);
    const double rho_ln = lmean(A.rho, B.rho);
    const double ibeta_ln = inv_lmean(ba, bb);
    const double ptil = (A.rho + B.rho) * rcp64(2.0 * (ba + bb));
    double va[3], Ba[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        va[k] = 0.5 * (A.v[k] + B.v[k]);
        Ba[k] = 0.5 * (A.B[k] + B.B[k]);
    }
    const double BB = dot3(A.B, B.B), v2a = 0.5 * (dot3(A.v, A.v) + dot3(B.v, B.v));
    const double vBa = dot3(A.v, A.B), vBb = dot3(B.v, B.B), B2a = dot3(A.B, A.B), B2b = dot3(B.B, B.B);
    const double Bna = sel2(d, A.B[0], A.B[1]), Bnb = sel2(d, B.B[0], B.B[1]);
    const double vna = sel2(d, A.v[0], A.v[1]), vnb = sel2(d, B.v[0], B.v[1]);
    const double psa = 0.5 * (A.psi + B.psi), Bnm = 0.5 * (Bna + Bnb);
    const double f0 = rho_ln * (0.5 * (vna + vnb));
    f[0] = f0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        f[1 + k] = fma(f0, va[k], fma(-0.5, fma(Bna, B.B[k], Bnb * A.B[k]), k == d ? fma(0.5, BB, ptil) : 0.0));
#pragma unroll
    for (int k = 0; k < 3; ++k)
        f[5 + k] = fma(0.5, fma(vna, A.B[k], fma(-A.v[k], Bna, fma(vnb, B.B[k], -B.v[k] * Bnb))),
                       k == d ? c_h * psa : 0.0);
    f[8] = c_h * Bnm;
    double fe = f0 * fma(0.5 * inv_gm1, ibeta_ln, -0.5 * v2a);
#pragma unroll
    for (int k = 0; k < 3; ++k) fe = fma(f[5 + k], Ba[k], fma(f[1 + k], va[k], fe));
    fe = fma(f[8], psa, fe);
    fe = fma(-0.25, fma(vna, B2a, vnb * B2b), fe);
    fe = fma(Bnm, 0.5 * (vBa + vBb), fe);
    fe = fma(-0.5 * c_h, fma(A.psi, Bna, B.psi * Bnb), fe);
    f[4] = fe;
}

// Fast magnetosonic speed in direction d.
__device__ __forceinline__ double mhd_cfast(int d, const PrimM &P, double gam)
{
    const double ir = rcp64(P.rho);
    const double a2 = gam * P.p * ir;
    const double b2 = (P.B[0] * P.B[0] + P.B[1] * P.B[1] + P.B[2] * P.B[2]) * ir;
    const double Bn = sel2(d, P.B[0], P.B[1]);
    return sqrt(0.5 * (a2 + b2 + sqrt((a2 + b2) * (a2 + b2) - 4.0 * a2 * Bn * Bn * ir)));
}

__device__ __forceinline__ void mhd_cons(const PrimM &P, double inv_gm1, double *u)
{
    u[0] = P.rho;
    double kin = 0.0, mag = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        u[1 + k] = P.rho * P.v[k];
        kin += P.v[k] * P.v[k];
        u[5 + k] = P.B[k];
        mag += P.B[k] * P.B[k];
    }
    u[4] = P.p * inv_gm1 + 0.5 * P.rho * kin + 0.5 * mag + 0.5 * P.psi * P.psi;
    u[8] = P.psi;
}

// Surface flux: EC, local Lax-Friedrichs (max |v_d| + c_f of both sides) or central.
__device__ __forceinline__ void mhd_flux_surface(int kind, int d, const PrimM &L, const PrimM &R, double gam,
                                                 double inv_gm1, double c_h, double *f)
{
#pragma clang fp contract(off)
    if (kind == PERRK_FLUX_EC) {
        mhd_flux_ec(d, L, R, inv_gm1, c_h, f);
        return;
    }
    double fl[MHD_V], fr[MHD_V];
    mhd_flux_phys(d, L, gam, inv_gm1, c_h, fl);
    mhd_flux_phys(d, R, gam, inv_gm1, c_h, fr);
#pragma unroll
    for (int k = 0; k < MHD_V; ++k) f[k] = 0.5 * (fl[k] + fr[k]);
    if (kind == PERRK_FLUX_LLF) {
        const double lam = fmax(fabs(sel2(d, L.v[0], L.v[1])) + mhd_cfast(d, L, gam),
                                fabs(sel2(d, R.v[0], R.v[1])) + mhd_cfast(d, R, gam));
        double ul[MHD_V], ur[MHD_V];
        mhd_cons(L, inv_gm1, ul);
        mhd_cons(R, inv_gm1, ur);
#pragma unroll
        for (int k = 0; k < MHD_V; ++k) f[k] -= 0.5 * lam * (ur[k] - ul[k]);
    }
}

// Entropy variables of s = -rho log(p rho^-gamma) with the MHD pressure.
__device__ __forceinline__ void mhd_entropy_vars(const double *u, double gam, double *w)
{
    const double rho = u[0], ir = 1.0 / rho;
    double m2 = 0.0, B2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        m2 += u[1 + k] * u[1 + k];
        B2 += u[5 + k] * u[5 + k];
    }
    const double p = (gam - 1.0) * (u[4] - 0.5 * m2 * ir - 0.5 * B2 - 0.5 * u[8] * u[8]);
    const double g1rp = (gam - 1.0) * rho / p;
    w[0] = gam - (flog(p) - gam * flog(rho)) - 0.5 * g1rp * m2 * ir * ir;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        w[1 + k] = g1rp * u[1 + k] * ir;
        w[5 + k] = g1rp * u[5 + k];
    }
    w[4] = -g1rp;
    w[8] = g1rp * u[8];
}

__device__ __forceinline__ double mhd_entropy_density(const double *u, double gam)
{
    double m2 = 0.0, B2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        m2 += u[1 + k] * u[1 + k];
        B2 += u[5 + k] * u[5 + k];
    }
    const double rho = u[0];
    const double p = (gam - 1.0) * (u[4] - 0.5 * m2 / rho - 0.5 * B2 - 0.5 * u[8] * u[8]);
    return -rho * (flog(p) - gam * flog(rho));
}

template <int KIND, bool ONE_DIR>
__global__ void __launch_bounds__(64 * PERRK_MAX_WPB) mhd_stage_kernel(const StageArgs a, const double *coef)
{
    constexpr int NPE = 16, V = MHD_V, NC = MHD_NC, EPW = 4, SLOT = mhd_slot<ONE_DIR>();
    constexpr int NFN = SG<2>::NFN, NPP = SG<2>::NPP, NPD = SG<2>::NPD, NLINE = SG<2>::NLINE;
    constexpr int FR = FaceRounds<2>::N;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *lds = reinterpret_cast<double *>(smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int eslot = wave * EPW + lane / NPE;
    const int node = lane % NPE;
    const int epb = (int)(blockDim.x >> 6) * EPW;
    const int li = xcd_block(blockIdx.x, gridDim.x) * epb + eslot;
    const bool valid = li < a.n_active;
    const int4 *ap = reinterpret_cast<const int4 *>(a.active);
    const uint32_t ai = (uint32_t)(valid ? li : a.n_active - 1);
    const int4 act = elt(ap, 2u * ai), act2 = elt(ap, 2u * ai + 1u);
    const int e = (int)((uint32_t)act.x & PERRK_NBR_MASK);
    const int lvl = (int)((uint32_t)act.x >> PERRK_NBR_SHIFT);
    double *slot = lds + (size_t)eslot * SLOT;
    const double gam = a.gam, gm1 = a.gm1, inv_gm1 = a.inv_gm1, c_h = a.c_h;
    int bad = 0;

    // ---- loads (as in the Euler kernel: own node, the neighbours' face nodes)
    double dt = 0.0, c1 = 0.0, cp = 0.0;
    if (KIND != SK_FIRST) {
        dt = elt(a.cs, (uint32_t)act.y).dt;
        c1 = elt(coef, (uint32_t)lvl);
        cp = elt(coef, (uint32_t)(PERRK_MAXR + lvl));
    }
    const size_t field = (size_t)a.nelem * NPE;
    NodeRaw<V, double> own;
    {
        const uint32_t o8 = ((uint32_t)e * NPE + node) * 8u;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            own.u[v] = bload<double>(field_rsrc<double>(a.U, v, field), o8);
            if (KIND != SK_FIRST) {
                own.k1[v] = bload<double>(field_rsrc<double>(a.K1, v, field), o8);
                own.kp[v] = bload<double>(field_rsrc<double>(a.Kp, v, field), o8);
            }
        }
    }
    double dacc[V];
    if constexpr (KIND == SK_LAST) {
        const uint32_t o8 = ((uint32_t)e * NPE + node) * 8u;
#pragma unroll
        for (int v = 0; v < V; ++v) dacc[v] = a.d_has ? bload<double>(field_rsrc<double>(a.d_out, v, field), o8) : 0.0;
    }
    FaceNode<2> F[FR];
    bool fv[FR];
    NodeRaw<V, double> nr[FR];
    double nc1[FR], ncp[FR];
#pragma unroll
    for (int r = 0; r < FR; ++r) {
        int nn;
        fv[r] = face_node<2>(r, lane, F[r], nn);
        const int f = 2 * F[r].d + F[r].side;
        const uint32_t w = (uint32_t)(f < 2 ? (f == 0 ? act.z : act.w) : (f == 2 ? act2.x : act2.y));
        const int nb = (int)(w & PERRK_NBR_MASK);
        nc1[r] = 0.0;
        ncp[r] = 0.0;
        if (KIND != SK_FIRST) {
            const int lv = (int)(w >> PERRK_NBR_SHIFT);
            nc1[r] = elt(coef, (uint32_t)lv);
            ncp[r] = elt(coef, (uint32_t)(PERRK_MAXR + lv));
        }
        const uint32_t o8 = ((uint32_t)nb * NPE + nn) * 8u;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            nr[r].u[v] = bload<double>(field_rsrc<double>(a.U, v, field), o8);
            if (KIND != SK_FIRST) {
                nr[r].k1[v] = bload<double>(field_rsrc<double>(a.K1, v, field), o8);
                nr[r].kp[v] = bload<double>(field_rsrc<double>(a.Kp, v, field), o8);
            }
        }
    }

    // ---- stage states
    double u[V];
    PrimM me, PN[FR];
    combine<V, double, KIND>(own, dt, c1, cp, u);
    make_prim_mhd(u, gm1, me, bad);
#pragma unroll
    for (int r = 0; r < FR; ++r) {
        double un[V];
        combine<V, double, KIND>(nr[r], dt, nc1[r], ncp[r], un);
        make_prim_mhd(un, gm1, PN[r], bad);
    }
    mhd_put(slot, node, me);
    wave_lds_sync();

    // ---- surface fluxes and face means of B_d and psi, lifted by +-6
#pragma unroll
    for (int r = 0; r < FR; ++r) {
        if (!fv[r]) continue;
        PrimM PO;
        mhd_get(slot, F[r].own, PO);
        const bool sd = F[r].side != 0;
        // minus / plus states selected value by value (registers, not addresses)
        PrimM L, R;
        L.rho = sd ? PO.rho : PN[r].rho;
        R.rho = sd ? PN[r].rho : PO.rho;
        L.p = sd ? PO.p : PN[r].p;
        R.p = sd ? PN[r].p : PO.p;
        L.psi = sd ? PO.psi : PN[r].psi;
        R.psi = sd ? PN[r].psi : PO.psi;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            L.v[k] = sd ? PO.v[k] : PN[r].v[k];
            R.v[k] = sd ? PN[r].v[k] : PO.v[k];
            L.B[k] = sd ? PO.B[k] : PN[r].B[k];
            R.B[k] = sd ? PN[r].B[k] : PO.B[k];
        }
        double fs[V];
        mhd_flux_surface(a.flux, F[r].d, L, R, gam, inv_gm1, c_h, fs);
        const double lift = sd ? 6.0 : -6.0;
        double *sf = slot + MHD_NQ * NPE;
#pragma unroll
        for (int v = 0; v < V; ++v) sf[v * NFN + F[r].q] = lift * fs[v];
        sf[9 * NFN + F[r].q] = lift * 0.5 * (sel2(F[r].d, L.B[0], L.B[1]) + sel2(F[r].d, R.B[0], R.B[1]));
        sf[10 * NFN + F[r].q] = lift * 0.5 * (L.psi + R.psi);
    }

    // ---- volume pairs (the two-point flux), and the gather:
    //      (2/h_d) [sum_m Dsplit f# + lifted face flux
    //               + Phi (sum_m Dsplit {B_d} + lifted face mean) + Phi_d (... psi)]
    // Two directions per phase (3 rounds of pairs, then both gathers), or one
    // direction at a time (ONE_DIR: pairs k = 0..3 of the direction on every lane,
    // then k = 4, 5 on lanes 0..31, its gather, then the other direction): the same
    // fluxes and sums in the same order.
    constexpr int VS = ONE_DIR ? NPD : NPP;  // pairs held per phase
    auto pair_flux = [&](int dd, int es, int l, int k) {
        int ta, tb;
        pair_pos(k, ta, tb);
        double *ps = lds + (size_t)(wave * EPW + es) * SLOT;
        PrimM A, B;
        mhd_get(ps, line_node<2>(dd, l, ta), A);
        mhd_get(ps, line_node<2>(dd, l, tb), B);
        double f[V];
        if (a.volume) {
            double fa[V], fb[V];
            mhd_flux_phys(dd, A, gam, inv_gm1, c_h, fa);
            mhd_flux_phys(dd, B, gam, inv_gm1, c_h, fb);
#pragma unroll
            for (int v = 0; v < V; ++v) f[v] = 0.5 * (fa[v] + fb[v]);
        } else {
            mhd_flux_ec(dd, A, B, inv_gm1, c_h, f);
        }
        double *vf = ps + MHD_NQ * NPE + NC * NFN;
        const int p = (ONE_DIR ? 0 : dd * NPD) + l * 6 + k;
#pragma unroll
        for (int v = 0; v < V; ++v) vf[v * VS + p] = f[v];
    };
    const ElemInfo ei = elt(a.elem, (uint32_t)e);
    double du[V];
#pragma unroll
    for (int v = 0; v < V; ++v) du[v] = 0.0;
    const double vB = me.v[0] * me.B[0] + me.v[1] * me.B[1] + me.v[2] * me.B[2];
    auto gather_dir = [&](int d) {
        const double *sf = slot + MHD_NQ * NPE;
        const double *vf = sf + NC * NFN;
        const int t = node_pos(d, node);
        const int l = node_line<2>(d, node);
        double acc[NC];
#pragma unroll
        for (int v = 0; v < NC; ++v) acc[v] = 0.0;
        const int pb = (ONE_DIR ? 0 : d * NPD) + l * 6;
        const int p1 = pb + pair_k<1>(t), p2 = pb + pair_k<2>(t), p3 = pb + pair_k<3>(t);
        const double w1 = dsplit_j<double, 1>(t), w2 = dsplit_j<double, 2>(t), w3 = dsplit_j<double, 3>(t);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            acc[v] += w1 * vf[v * VS + p1];
            acc[v] += w2 * vf[v * VS + p2];
            acc[v] += w3 * vf[v * VS + p3];
        }
        // pair means of B_d and psi with the partners (t + j) & 3 (a symmetric
        // sum, so it does not matter which node of the pair it is formed on)
        const double *q1 = slot + line_node<2>(d, l, (t + 1) & 3) * MHD_NQ;
        const double *q2 = slot + line_node<2>(d, l, (t + 2) & 3) * MHD_NQ;
        const double *q3 = slot + line_node<2>(d, l, (t + 3) & 3) * MHD_NQ;
        const double bt = sel2(d, me.B[0], me.B[1]);
        acc[9] += w1 * (0.5 * (bt + q1[5 + d]));
        acc[9] += w2 * (0.5 * (bt + q2[5 + d]));
        acc[9] += w3 * (0.5 * (bt + q3[5 + d]));
        acc[10] += w1 * (0.5 * (me.psi + q1[8]));
        acc[10] += w2 * (0.5 * (me.psi + q2[8]));
        acc[10] += w3 * (0.5 * (me.psi + q3[8]));
        if (t == 0 || t == 3) {
            const int q = (2 * d + (t == 3 ? 1 : 0)) * NLINE + l;
#pragma unroll
            for (int v = 0; v < NC; ++v) acc[v] += sf[v * NFN + q];
        }
        // non-conservative terms of the node's own state
        const double vn = sel2(d, me.v[0], me.v[1]);
        acc[1] += me.B[0] * acc[9];
        acc[2] += me.B[1] * acc[9];
        acc[3] += me.B[2] * acc[9];
        acc[4] += vB * acc[9] + vn * me.psi * acc[10];
        acc[5] += me.v[0] * acc[9];
        acc[6] += me.v[1] * acc[9];
        acc[7] += me.v[2] * acc[9];
        acc[8] += vn * acc[10];
        const double h = d == 0 ? ei.metric[0] : ei.metric[1];
#pragma unroll
        for (int v = 0; v < V; ++v) du[v] += h * acc[v];
    };
    if constexpr (ONE_DIR) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            pair_flux(d, lane >> 4, (lane >> 2) & 3, lane & 3);
            if (lane < 32) pair_flux(d, lane >> 3, (lane >> 1) & 3, 4 + (lane & 1));
            wave_lds_sync();
            gather_dir(d);
            wave_lds_sync();
        }
    } else {
#pragma unroll
        for (int rd = 0; rd < PairRounds<2, 2>::N; ++rd) {
            int es, dd, l, k;
            pair_of<2, 2>(rd, lane, es, dd, l, k);
            pair_flux(dd, es, l, k);
        }
        wave_lds_sync();
        gather_dir(0);
        gather_dir(1);
    }

    double k[V];
#pragma unroll
    for (int v = 0; v < V; ++v) k[v] = -du[v];
    if (valid) {
        const uint32_t o8 = ((uint32_t)e * NPE + node) * 8u;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (KIND == SK_LAST) {
                double dv = a.bs * k[v];
                if (a.bsm1 != 0.0) dv += a.bsm1 * own.kp[v];
                if (a.b1 != 0.0) dv += a.b1 * own.k1[v];
                if (a.d_has) dv += dacc[v];
                bstore<double>(dv, field_rsrc<double>(a.d_out, v, field), o8);
            } else {
                bstore<double>(k[v], field_rsrc<double>(a.Kout, v, field), o8);
                if (a.acc_mode) {
                    double dv = a.b_acc * k[v];
                    if (a.acc_mode == 2) dv += bload<double>(field_rsrc<double>(a.d_out, v, field), o8);
                    bstore<double>(dv, field_rsrc<double>(a.d_out, v, field), o8);
                }
            }
        }
    }
    if (a.ep_partial != nullptr) {
        double w[V];
        mhd_entropy_vars(u, gam, w);
        double dot = 0.0;
#pragma unroll
        for (int v = 0; v < V; ++v) dot += w[v] * k[v];
        double sm = node_weight<2>(node) * dot;
#pragma unroll
        for (int off = NPE / 2; off >= 1; off >>= 1) sm += __shfl_xor(sm, off);
        if (valid && node == 0) a.ep_partial[e] = ei.jac * sm;
    }
    if (bad && valid) atomicOr(a.err, bad);
}

// ---------------------------------------------------------------- Navier-Stokes-Fourier (BR1), 2D
// Viscous terms added to the Euler equations in double precision: gradients of
// q = (rho, v_x, v_y, T), T = p / rho, by the strong-form derivative with face
// means (BR1), then the divergence of the viscous flux (Stokes stress, heat
// conductivity kappa = gamma mu / ((gamma-1) Pr)) in the same form.  The
// full-derivative row of a node at position t is Dsplit/2 off the diagonal and
// D_tt = -3, 0, 0, 3 on it.  The viscous-shock set-up (one case) replaces the
// two x ends of the mesh by boundaries: exact inflow / free outflow for the
// inviscid flux and moving isothermal walls (exact velocity and temperature)
// for the viscous terms, at the stage time t_n + c_i dt.
constexpr int NS_NQ = 4;  // q per node
constexpr int NS_SLOT = NS_NQ * 16 + 8 * 16 + 4 * (SG<2>::NFN + SG<2>::NPP) + 6 * 16 + 3 * SG<2>::NFN;
// slot layout (doubles): prims [node][4] (rho, v_x, v_y, p) | gradients g[8][node] |
// inviscid sf[4][NFN], vf[4][NPP] | viscous node fluxes fvn[6][node] (dir, m_x, m_y, E) |
// lifted viscous face terms sfv[3][NFN]
constexpr int NS_OFF_G = NS_NQ * 16, NS_OFF_SF = NS_OFF_G + 8 * 16, NS_OFF_VF = NS_OFF_SF + 4 * SG<2>::NFN,
              NS_OFF_FVN = NS_OFF_VF + 4 * SG<2>::NPP, NS_OFF_SFV = NS_OFF_FVN + 6 * 16;
constexpr int NS_GRAD_SLOT = NS_NQ * 16 + NS_NQ * SG<2>::NFN;  // gradient kernel: q [node][4] | lifted sq[4][NFN]

// Exact viscous shock (rho_0 = 1, shock speed 1, Ma = 2/sqrt(3 - gamma),
// l = 2 gamma (4/3 mu)/(gamma + 1)): primitive rho, v_x, p at (x, t).
__device__ __forceinline__ void viscous_shock(double x, double t, double gam, double mu, double &rho, double &vx,
                                              double &p)
{
    const double Ma2 = 4.0 / (3.0 - gam);
    const double p0 = 1.0 / (gam * Ma2);
    const double l = 2.0 * gam * (4.0 / 3.0 * mu) / (gam + 1.0);
    const double chi = 2.0 * exp((x - t) / (2.0 * l));
    const double w = 1.0 + (1.0 - sqrt(1.0 + 2.0 * chi * chi)) / (2.0 * chi * chi);
    rho = 1.0 / w;
    vx = 1.0 - w;
    p = p0 / w * (1.0 + 0.5 * (gam - 1.0) * Ma2 * (1.0 - w * w));
}

// Viscous flux in direction d (components m_x, m_y, E; the mass component is 0)
// from the velocity and the gradients g[dir * 4 + k] of q.
__device__ __forceinline__ void ns_vflux(int d, double vx, double vy, const double *g, double mu, double kappa,
                                         double *f)
{
    const double div = g[1] + g[4 + 2];
    const double txx = mu * (2.0 * g[1] - 2.0 / 3.0 * div);
    const double tyy = mu * (2.0 * g[4 + 2] - 2.0 / 3.0 * div);
    const double txy = mu * (g[4 + 1] + g[2]);
    const double tn0 = d == 0 ? txx : txy, tn1 = d == 0 ? txy : tyy;
    f[0] = tn0;
    f[1] = tn1;
    f[2] = vx * tn0 + vy * tn1 + kappa * (d == 0 ? g[3] : g[4 + 3]);
}

__device__ __forceinline__ double dfull_diag(int t) { return t == 0 ? -3.0 : (t == 3 ? 3.0 : 0.0); }

// Shared load phase of the two Navier-Stokes kernels: the active entry, the
// stage coefficients, the own node's raw data and the neighbour's at the lane's
// face node (the neighbour words and the boundary flags come with the entry).
struct NsLoad {
    int e, lvl, cs;
    uint32_t bcf;  // bit 0: left x face is a boundary, bit 1: right x face
    double dt, c1, cp;
    NodeRaw<4, double> own, nr;
    double nc1, ncp;
    FaceNode<2> F;
    bool fv;
    int nb, nn;
};

template <int KIND>
__device__ __forceinline__ void ns_load(const StageArgs &a, const double *coef, uint32_t ai, int lane, int node,
                                        NsLoad &L)
{
    constexpr int NPE = 16;
    const int4 *ap = reinterpret_cast<const int4 *>(a.active);
    const int4 act = elt(ap, 2u * ai), act2 = elt(ap, 2u * ai + 1u);
    L.e = (int)((uint32_t)act.x & PERRK_NBR_MASK);
    L.lvl = (int)((uint32_t)act.x >> PERRK_NBR_SHIFT);
    L.cs = act.y;
    L.bcf = (uint32_t)act2.z;
    L.dt = L.c1 = L.cp = 0.0;
    if (KIND != SK_FIRST) {
        L.dt = elt(a.cs, (uint32_t)L.cs).dt;
        L.c1 = elt(coef, (uint32_t)L.lvl);
        L.cp = elt(coef, (uint32_t)(PERRK_MAXR + L.lvl));
    }
    const size_t field = (size_t)a.nelem * NPE;
    const uint32_t o8 = ((uint32_t)L.e * NPE + node) * 8u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        L.own.u[v] = bload<double>(field_rsrc<double>(a.U, v, field), o8);
        if (KIND != SK_FIRST) {
            L.own.k1[v] = bload<double>(field_rsrc<double>(a.K1, v, field), o8);
            L.own.kp[v] = bload<double>(field_rsrc<double>(a.Kp, v, field), o8);
        }
    }
    L.fv = face_node<2>(0, lane, L.F, L.nn);
    const int f = 2 * L.F.d + L.F.side;
    const uint32_t w = (uint32_t)(f < 2 ? (f == 0 ? act.z : act.w) : (f == 2 ? act2.x : act2.y));
    L.nb = (int)(w & PERRK_NBR_MASK);
    L.nc1 = L.ncp = 0.0;
    if (KIND != SK_FIRST) {
        const int lv = (int)(w >> PERRK_NBR_SHIFT);
        L.nc1 = elt(coef, (uint32_t)lv);
        L.ncp = elt(coef, (uint32_t)(PERRK_MAXR + lv));
    }
    const uint32_t n8 = ((uint32_t)L.nb * NPE + L.nn) * 8u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        L.nr.u[v] = bload<double>(field_rsrc<double>(a.U, v, field), n8);
        if (KIND != SK_FIRST) {
            L.nr.k1[v] = bload<double>(field_rsrc<double>(a.K1, v, field), n8);
            L.nr.kp[v] = bload<double>(field_rsrc<double>(a.Kp, v, field), n8);
        }
    }
}

// True when the lane's face is an x boundary of the viscous-shock mesh.
__device__ __forceinline__ bool ns_boundary(const NsLoad &L)
{
    return L.F.d == 0 && (L.bcf & (L.F.side ? 2u : 1u)) != 0u;
}

// Gradient pass of one stage (every element): g = (2/h_d) [D q + lifted (q* - q)].
template <int KIND>
__global__ void __launch_bounds__(64 * PERRK_MAX_WPB) ns_grad_kernel(const StageArgs a, const double *coef)
{
    constexpr int NPE = 16, EPW = 4, NFN = SG<2>::NFN, NLINE = SG<2>::NLINE, SLOT = NS_GRAD_SLOT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *lds = reinterpret_cast<double *>(smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int eslot = wave * EPW + lane / NPE;
    const int node = lane % NPE;
    const int epb = (int)(blockDim.x >> 6) * EPW;
    const int li = xcd_block(blockIdx.x, gridDim.x) * epb + eslot;
    const bool valid = li < a.n_active;
    double *slot = lds + (size_t)eslot * SLOT;
    NsLoad L;
    ns_load<KIND>(a, coef, (uint32_t)(valid ? li : a.n_active - 1), lane, node, L);
    int bad = 0;
    double u[4], un[4];
    combine<4, double, KIND>(L.own, L.dt, L.c1, L.cp, u);
    combine<4, double, KIND>(L.nr, L.dt, L.nc1, L.ncp, un);
    Prim<double, 2> me, pn;
    make_prim<double, 2>(u, a.gm1, me, bad);
    make_prim<double, 2>(un, a.gm1, pn, bad);
    double *q = slot + node * 4;
    q[0] = me.rho;
    q[1] = me.v[0];
    q[2] = me.v[1];
    q[3] = me.p * rcp64(me.rho);
    wave_lds_sync();
    if (L.fv) {
        const double *qo = slot + L.F.own * 4;
        double qs[4];
        if (ns_boundary(L)) {
            // moving isothermal wall: exact velocity and temperature, the trace's density
            const double tt = elt(a.cs, (uint32_t)L.cs).t + a.c_stage * L.dt;
            double r, vx, p;
            viscous_shock(L.F.side ? a.x_hi : a.x_lo, tt, a.gam, a.mu, r, vx, p);
            qs[0] = qo[0];
            qs[1] = vx;
            qs[2] = 0.0;
            qs[3] = p / r;
        } else {
            qs[0] = 0.5 * (qo[0] + pn.rho);
            qs[1] = 0.5 * (qo[1] + pn.v[0]);
            qs[2] = 0.5 * (qo[2] + pn.v[1]);
            qs[3] = 0.5 * (qo[3] + pn.p * rcp64(pn.rho));
        }
        const double lift = L.F.side ? 6.0 : -6.0;
        double *sq = slot + 4 * NPE;
#pragma unroll
        for (int k = 0; k < 4; ++k) sq[k * NFN + L.F.q] = lift * (qs[k] - qo[k]);
    }
    wave_lds_sync();
    if (!valid) return;
    const ElemInfo ei = elt(a.elem, (uint32_t)L.e);
    const size_t field = (size_t)a.nelem * NPE;
    const uint32_t o8 = ((uint32_t)L.e * NPE + node) * 8u;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const int t = node_pos(d, node), l = node_line<2>(d, node);
        const double *q1 = slot + line_node<2>(d, l, (t + 1) & 3) * 4;
        const double *q2 = slot + line_node<2>(d, l, (t + 2) & 3) * 4;
        const double *q3 = slot + line_node<2>(d, l, (t + 3) & 3) * 4;
        const double *qt = slot + node * 4;
        const double w1 = 0.5 * dsplit_j<double, 1>(t), w2 = 0.5 * dsplit_j<double, 2>(t);
        const double w3 = 0.5 * dsplit_j<double, 3>(t), w0 = dfull_diag(t);
        const double h = d == 0 ? ei.metric[0] : ei.metric[1];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double acc = w0 * qt[k] + w1 * q1[k] + w2 * q2[k] + w3 * q3[k];
            if (t == 0 || t == 3) acc += slot[4 * NPE + k * NFN + (2 * d + (t == 3 ? 1 : 0)) * NLINE + l];
            bstore<double>(h * acc, field_rsrc<double>(a.grad, d * 4 + k, field), o8);
        }
    }
    if (bad) atomicOr(a.err, bad);
}

// Stage kernel with viscous terms (double precision, 2D): inviscid part with the
// EC or a dissipative surface flux and EC flux differencing or the weak form,
// plus the BR1 divergence of the viscous flux.
template <int KIND>
__global__ void __launch_bounds__(64 * PERRK_MAX_WPB) ns_stage_kernel(const StageArgs a, const double *coef)
{
    constexpr int NPE = 16, EPW = 4, NFN = SG<2>::NFN, NPP = SG<2>::NPP, NPD = SG<2>::NPD, NLINE = SG<2>::NLINE;
    constexpr int SLOT = NS_SLOT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *lds = reinterpret_cast<double *>(smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int eslot = wave * EPW + lane / NPE;
    const int node = lane % NPE;
    const int epb = (int)(blockDim.x >> 6) * EPW;
    const int li = xcd_block(blockIdx.x, gridDim.x) * epb + eslot;
    const bool valid = li < a.n_active;
    double *slot = lds + (size_t)eslot * SLOT;
    const double gam = a.gam, inv_gm1 = a.inv_gm1;
    const double kappa = a.gam * a.mu / ((a.gam - 1.0) * a.prandtl);
    NsLoad L;
    ns_load<KIND>(a, coef, (uint32_t)(valid ? li : a.n_active - 1), lane, node, L);
    const size_t field = (size_t)a.nelem * NPE;
    const uint32_t o8 = ((uint32_t)L.e * NPE + node) * 8u, n8 = ((uint32_t)L.nb * NPE + L.nn) * 8u;
    double go[8], gn[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        go[k] = bload<double>(field_rsrc<double>(a.grad, k, field), o8);
        gn[k] = bload<double>(field_rsrc<double>(a.grad, k, field), n8);
    }
    double dacc[4];
    if constexpr (KIND == SK_LAST) {
#pragma unroll
        for (int v = 0; v < 4; ++v) dacc[v] = a.d_has ? bload<double>(field_rsrc<double>(a.d_out, v, field), o8) : 0.0;
    }
    int bad = 0;
    double u[4], un[4];
    combine<4, double, KIND>(L.own, L.dt, L.c1, L.cp, u);
    combine<4, double, KIND>(L.nr, L.dt, L.nc1, L.ncp, un);
    Prim<double, 2> me, pn;
    make_prim<double, 2>(u, a.gm1, me, bad);
    make_prim<double, 2>(un, a.gm1, pn, bad);
    {
        double *q = slot + node * 4;
        q[0] = me.rho;
        q[1] = me.v[0];
        q[2] = me.v[1];
        q[3] = me.p;
        double *g = slot + NS_OFF_G;
#pragma unroll
        for (int k = 0; k < 8; ++k) g[k * NPE + node] = go[k];
        // viscous flux of the own node in both directions
        double fx[3], fy[3];
        ns_vflux(0, me.v[0], me.v[1], go, a.mu, kappa, fx);
        ns_vflux(1, me.v[0], me.v[1], go, a.mu, kappa, fy);
        double *fvn = slot + NS_OFF_FVN;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            fvn[c * NPE + node] = fx[c];
            fvn[(3 + c) * NPE + node] = fy[c];
        }
    }
    wave_lds_sync();

    // ---- faces: inviscid flux (ghost states at the x ends) and viscous face terms
    if (L.fv) {
        Prim<double, 2> PO;
        {
            const double *q = slot + L.F.own * 4;
            PO.rho = q[0];
            PO.v[0] = q[1];
            PO.v[1] = q[2];
            PO.p = q[3];
            PO.beta = PO.rho * rcp64(PO.p);
        }
        const bool bnd = ns_boundary(L);
        const double tt = elt(a.cs, (uint32_t)L.cs).t + a.c_stage * L.dt;
        double rw = 0.0, vw = 0.0, pw = 1.0;
        if (bnd) viscous_shock(L.F.side ? a.x_hi : a.x_lo, tt, gam, a.mu, rw, vw, pw);
        Prim<double, 2> PG = pn;
        if (bnd) {
            if (L.F.side) {
                PG = PO;  // free outflow: the trace itself
            } else {      // inflow: the exact state
                PG.rho = rw;
                PG.v[0] = vw;
                PG.v[1] = 0.0;
                PG.p = pw;
                PG.beta = rw * rcp64(pw);
            }
        }
        const bool sd = L.F.side != 0;
        Prim<double, 2> A, B;
        A.rho = sd ? PO.rho : PG.rho;
        B.rho = sd ? PG.rho : PO.rho;
        A.p = sd ? PO.p : PG.p;
        B.p = sd ? PG.p : PO.p;
        A.beta = sd ? PO.beta : PG.beta;
        B.beta = sd ? PG.beta : PO.beta;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            A.v[k] = sd ? PO.v[k] : PG.v[k];
            B.v[k] = sd ? PG.v[k] : PO.v[k];
        }
        double fs[4];
        if (a.flux != PERRK_FLUX_EC) flux_diss<double, 2>(a.flux, L.F.d, A, B, gam, inv_gm1, fs);
        else flux_ec<double, 2>(L.F.d, A, B, inv_gm1, fs);
        const double lift = sd ? 6.0 : -6.0;
        double *sf = slot + NS_OFF_SF;
#pragma unroll
        for (int v = 0; v < 4; ++v) sf[v * NFN + L.F.q] = lift * fs[v];
        // viscous: F* - F_own at the own face node
        const double *fvn = slot + NS_OFF_FVN + (L.F.d == 0 ? 0 : 3 * NPE);
        double fo[3], fstar[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) fo[c] = fvn[c * NPE + L.F.own];
        if (bnd) {
            double gown[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) gown[k] = slot[NS_OFF_G + k * NPE + L.F.own];
            ns_vflux(L.F.d, vw, 0.0, gown, a.mu, kappa, fstar);
        } else {
            double fn[3];
            ns_vflux(L.F.d, pn.v[0], pn.v[1], gn, a.mu, kappa, fn);
#pragma unroll
            for (int c = 0; c < 3; ++c) fstar[c] = 0.5 * (fo[c] + fn[c]);
        }
        double *sfv = slot + NS_OFF_SFV;
#pragma unroll
        for (int c = 0; c < 3; ++c) sfv[c * NFN + L.F.q] = lift * (fstar[c] - fo[c]);
    }

    // ---- inviscid pair fluxes (EC or central)
#pragma unroll
    for (int rd = 0; rd < PairRounds<2, 2>::N; ++rd) {
        int es, dd, l, k;
        pair_of<2, 2>(rd, lane, es, dd, l, k);
        int ta, tb;
        pair_pos(k, ta, tb);
        double *ps = lds + (size_t)(wave * EPW + es) * SLOT;
        Prim<double, 2> A, B;
        {
            const double *qa = ps + line_node<2>(dd, l, ta) * 4, *qb = ps + line_node<2>(dd, l, tb) * 4;
            A.rho = qa[0];
            A.v[0] = qa[1];
            A.v[1] = qa[2];
            A.p = qa[3];
            A.beta = A.rho * rcp64(A.p);
            B.rho = qb[0];
            B.v[0] = qb[1];
            B.v[1] = qb[2];
            B.p = qb[3];
            B.beta = B.rho * rcp64(B.p);
        }
        double f[4];
        if (a.volume) flux_central<double, 2>(dd, A, B, inv_gm1, f);
        else flux_ec<double, 2>(dd, A, B, inv_gm1, f);
        double *vf = ps + NS_OFF_VF;
        const int p = dd * NPD + l * 6 + k;
#pragma unroll
        for (int v = 0; v < 4; ++v) vf[v * NPP + p] = f[v];
    }
    wave_lds_sync();

    // ---- gather: inviscid (split form) and viscous (full derivative) per direction
    const ElemInfo ei = elt(a.elem, (uint32_t)L.e);
    double k[4] = {0.0, 0.0, 0.0, 0.0};
    {
        const double *sf = slot + NS_OFF_SF, *vf = slot + NS_OFF_VF;
        const double *fvn = slot + NS_OFF_FVN, *sfv = slot + NS_OFF_SFV;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const int t = node_pos(d, node), l = node_line<2>(d, node);
            const int pb = d * NPD + l * 6;
            const int p1 = pb + pair_k<1>(t), p2 = pb + pair_k<2>(t), p3 = pb + pair_k<3>(t);
            const double w1 = dsplit_j<double, 1>(t), w2 = dsplit_j<double, 2>(t), w3 = dsplit_j<double, 3>(t);
            const int qf = (2 * d + (t == 3 ? 1 : 0)) * NLINE + l;
            const double h = d == 0 ? ei.metric[0] : ei.metric[1];
            double ai[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                ai[v] = w1 * vf[v * NPP + p1] + w2 * vf[v * NPP + p2] + w3 * vf[v * NPP + p3];
                if (t == 0 || t == 3) ai[v] += sf[v * NFN + qf];
                k[v] -= h * ai[v];
            }
            const int n1 = line_node<2>(d, l, (t + 1) & 3), n2 = line_node<2>(d, l, (t + 2) & 3);
            const int n3 = line_node<2>(d, l, (t + 3) & 3);
            const double *fd = fvn + (d == 0 ? 0 : 3 * NPE);
            const double w0 = dfull_diag(t);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double av = w0 * fd[c * NPE + node] + 0.5 * (w1 * fd[c * NPE + n1] + w2 * fd[c * NPE + n2] +
                                                             w3 * fd[c * NPE + n3]);
                if (t == 0 || t == 3) av += sfv[c * NFN + qf];
                k[1 + c] += h * av;
            }
        }
    }

    if (valid) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (KIND == SK_LAST) {
                double dv = a.bs * k[v];
                if (a.bsm1 != 0.0) dv += a.bsm1 * L.own.kp[v];
                if (a.b1 != 0.0) dv += a.b1 * L.own.k1[v];
                if (a.d_has) dv += dacc[v];
                bstore<double>(dv, field_rsrc<double>(a.d_out, v, field), o8);
            } else {
                bstore<double>(k[v], field_rsrc<double>(a.Kout, v, field), o8);
                if (a.acc_mode) {
                    double dv = a.b_acc * k[v];
                    if (a.acc_mode == 2) dv += bload<double>(field_rsrc<double>(a.d_out, v, field), o8);
                    bstore<double>(dv, field_rsrc<double>(a.d_out, v, field), o8);
                }
            }
        }
    }
    if (a.ep_partial != nullptr) {
        double w[4];
        entropy_vars<2>(u, gam, w);
        double dot = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) dot += w[v] * k[v];
        double sm = node_weight<2>(node) * dot;
#pragma unroll
        for (int off = NPE / 2; off >= 1; off >>= 1) sm += __shfl_xor(sm, off);
        if (valid && node == 0) a.ep_partial[L.e] = ei.jac * sm;
    }
    if (bad && valid) atomicOr(a.err, bad);
}

// ---------------------------------------------------------------- reductions
// Sum of NC per-element partials over [b, e) by PERRK_RED_THREADS threads in a
// fixed order (strided sequential sums, then a fixed tree).  Result in out on
// every thread.  Each thread issues the loads of CS_AHEAD of its elements before
// adding them (in the same order), so that a large case is not summed at one
// memory latency per element.
constexpr int CS_AHEAD = 8;

template <int NC>
__device__ __forceinline__ void case_sum(const double *part, int stride, int64_t b, int64_t e,
                                         double *out)
{
    __shared__ double red[NC][PERRK_RED_THREADS];
    const int t = threadIdx.x;
    constexpr int64_t T = PERRK_RED_THREADS;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    int64_t i = b + t;
    for (; i + (CS_AHEAD - 1) * T < e; i += CS_AHEAD * T) {
        double x[CS_AHEAD][NC];
#pragma unroll
        for (int k = 0; k < CS_AHEAD; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) x[k][c] = part[(size_t)(i + k * T) * stride + c];
#pragma unroll
        for (int k = 0; k < CS_AHEAD; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] += x[k][c];
    }
    for (; i < e; i += T) {
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

// The same for ideal GLM-MHD (nine variables): the pressure change gains
//   -(gamma-1) [(B.dB + |dB|^2/2) + (psi dpsi + dpsi^2/2)],
// and w' gains the components (gamma-1) rho' B' / p' and (gamma-1) rho' psi' / p'.
__device__ __forceinline__ void relax_node_mhd(const double *u, const double *dv, double g, double dt, double gam,
                                               double &ds, double &wd)
{
#pragma clang fp contract(off)
    const double rho = u[0];
    double du[MHD_V];
#pragma unroll
    for (int v = 0; v < MHD_V; ++v) du[v] = g * dt * dv[v];
    const double drho = du[0], rho1 = rho + drho;
    const double ir = 1.0 / rho, ir1 = 1.0 / rho1;
    double mdm = 0.0, dm2 = 0.0, m2 = 0.0, B2 = 0.0, BdB = 0.0, dB2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        mdm += u[1 + k] * du[1 + k];
        dm2 += du[1 + k] * du[1 + k];
        m2 += u[1 + k] * u[1 + k];
        B2 += u[5 + k] * u[5 + k];
        BdB += u[5 + k] * du[5 + k];
        dB2 += du[5 + k] * du[5 + k];
    }
    const double g1 = gam - 1.0;
    const double p = g1 * (u[4] - 0.5 * m2 * ir - 0.5 * B2 - 0.5 * u[8] * u[8]);
    const double dp = g1 * (du[4] - (mdm + 0.5 * dm2) * ir1 + 0.5 * drho * m2 * ir * ir1 - (BdB + 0.5 * dB2)
                            - (u[8] * du[8] + 0.5 * du[8] * du[8]));
    const double p1 = p + dp;
    const double lp = log1p_small(dp / p), lr = log1p_small(drho * ir);
    const double sth0 = flog(p) - gam * flog(rho);
    const double sth1 = sth0 + lp - gam * lr;
    ds = -drho * sth1 - rho * (lp - gam * lr);
    const double ip1 = 1.0 / p1;
    const double m12 = m2 + 2.0 * mdm + dm2;
    const double g1rp = g1 * rho1 * ip1;
    double dot = (gam - sth1 - 0.5 * g1 * m12 * ir1 * ip1) * dv[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dot += g1 * (u[1 + k] + du[1 + k]) * ip1 * dv[1 + k];
        dot += g1rp * (u[5 + k] + du[5 + k]) * dv[5 + k];
    }
    dot += -g1rp * dv[4];
    dot += g1rp * (u[8] + du[8]) * dv[8];
    wd = dt * dot;
}

// Nodes, fields and elements per wavefront of a system (SYS 0: Euler, 1: GLM-MHD in 2D).
template <int DIM, int SYS>
struct Sys {
    static constexpr int NPE = Geo<DIM>::NPE, EPW = Geo<DIM>::EPW;
    static constexpr int V = SYS == 1 ? MHD_V : Geo<DIM>::V;
};

// Per-element residual partials: J sum q Delta s at gamma, J sum q w(u + gamma dt d) . dt d,
// J sum q Delta s at gamma_b (only while opening a bracket), sum |d|.  Node
// lane of element e of case C (jac: the element's Jacobian); u, dv: the node's
// U_n and d, loaded by load() where the case needs an evaluation (a no-op where
// the caller loaded them already).
template <int DIM, int SYS, typename Load>
__device__ __forceinline__ void relax_finish(const CaseState &C, double jac, double *partial, int64_t e, int node,
                                             bool valid, double gam, const double *u, const double *dv, Load load)
{
    constexpr int NPE = Sys<DIM, SYS>::NPE, V = Sys<DIM, SYS>::V;
    const int st = C.state;
    const bool live = valid && st != RS_DONE && st != RS_FALLBACK && st != RS_EVAL1;
    const bool eval1 = valid && st == RS_EVAL1;
    double sr = 0.0, srp = 0.0, srb = 0.0, sabs = 0.0;
    if (live || eval1) {
        const double g = eval1 ? 1.0 : C.gamma;
        const double dt = C.dt;
        load();
#pragma unroll
        for (int v = 0; v < V; ++v) sabs += fabs(dv[v]);
        const double q = node_weight<DIM>(node);
        double ds, wd;
        if constexpr (SYS == 1) relax_node_mhd(u, dv, g, dt, gam, ds, wd);
        else relax_node<DIM>(u, dv, g, dt, gam, ds, wd);
        sr = q * ds;
        srp = q * wd;
        if (!eval1 && st == RS_BIS_INIT) {
            if constexpr (SYS == 1) relax_node_mhd(u, dv, C.gamma_b, dt, gam, ds, wd);
            else relax_node<DIM>(u, dv, C.gamma_b, dt, gam, ds, wd);
            srb = q * ds;
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
        pp[0] = jac * sr;
        pp[1] = jac * srp;
        pp[2] = jac * srb;
        pp[3] = sabs;
    }
}

template <int DIM, int SYS>
__device__ __forceinline__ void relax_load(const double *U, const double *dd, int64_t nelem, int64_t e, int node,
                                           double *u, double *dv)
{
    constexpr int NPE = Sys<DIM, SYS>::NPE, V = Sys<DIM, SYS>::V;
    const size_t field = (size_t)nelem * NPE;
    const uint32_t o8 = ((uint32_t)e * NPE + (uint32_t)node) * 8u;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        u[v] = bload<double>(field_rsrc<double>(U, v, field), o8);
        dv[v] = bload<double>(field_rsrc<double>(dd, v, field), o8);
    }
}

// One element per call.  PRELOAD (the launched passes, whose blocks hold a case
// being solved): the node loads go out with the element and case-state loads;
// otherwise they are issued only where the case needs an evaluation.
template <int DIM, int SYS, bool PRELOAD = false>
__device__ __forceinline__ void relax_element(const double *U, const double *dd, const ElemInfo *elem,
                                              const CaseState *cs, double *partial, int64_t nelem,
                                              double gam, int64_t e, int node, bool valid)
{
    constexpr int V = Sys<DIM, SYS>::V;
    const ElemInfo ei = elem[e];
    double u[V], dv[V];
    if constexpr (PRELOAD) relax_load<DIM, SYS>(U, dd, nelem, e, node, u, dv);
    relax_finish<DIM, SYS>(cs[ei.case_id], ei.jac, partial, e, node, valid, gam, u, dv, [&]() {
        if constexpr (!PRELOAD) relax_load<DIM, SYS>(U, dd, nelem, e, node, u, dv);
    });
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

// Per-case sums of the prepare kernel over a case of more than PERRK_RED_CHUNK
// elements: the case is cut into chunks of PERRK_RED_CHUNK elements (the last one
// shorter), one workgroup sums each chunk in the fixed order of case_sum, and
// the prepare kernel adds the chunk sums in chunk order.  A case of at most
// PERRK_RED_CHUNK elements is summed as before, over its elements.
// chunk_sums[k][j]: the sum of ep_j over chunk k (j < PERRK_MAXB, the ones the
// phase reduces), [k][PERRK_MAXB + i]: of the fused residual partial i (phase 2).
constexpr int PREP_NV = PERRK_MAXB + 4;

__global__ void __launch_bounds__(PERRK_RED_THREADS)
prepare_chunks_kernel(const int64_t *chunk_range, const double *ep, int64_t nelem, RelaxParams rp, int phase,
                      const double *rx_partial, double *chunk_sums)
{
    const int k = blockIdx.x;
    const int64_t b = chunk_range[2 * k], e = chunk_range[2 * k + 1];
    double *out = chunk_sums + (size_t)k * PREP_NV;
    const int j0 = phase == 2 ? rp.nb_pre : 0, j1 = phase == 1 ? rp.nb_pre : rp.nb;
    for (int j = j0; j < j1; ++j) {
        double o[1];
        case_sum<1>(ep + (size_t)j * nelem, 1, b, e, o);
        if (threadIdx.x == 0) out[j] = o[0];
    }
    if (phase == 2) {
        double S[4];
        case_sum<4>(rx_partial, 4, b, e, S);
        if (threadIdx.x == 0)
            for (int i = 0; i < 4; ++i) out[PERRK_MAXB + i] = S[i];
    }
}

// One per-case sum of the prepare kernel: over the case's elements [b, e), or
// (a case cut into the chunks [k0, k1)) over the chunk sums in chunk order.
// Component i of the NC-wide sum is chunk entry v0 + i.
template <int NC>
__device__ __forceinline__ void prep_sum(const double *part, int stride, int64_t b, int64_t e, int k0, int k1,
                                         const double *chunk_sums, int v0, double *out)
{
    if (k1 - k0 < 2) {
        case_sum<NC>(part, stride, b, e, out);
        return;
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        double acc = chunk_sums[(size_t)k0 * PREP_NV + v0 + i];
        for (int k = k0 + 1; k < k1; ++k) acc += chunk_sums[(size_t)k * PREP_NV + v0 + i];
        out[i] = acc;
    }
}

// Residual passes of a step that find every case solved leave at once.  The
// kernel that last updated the solver states before a pass (the prepare kernel,
// then each finalize) raises the pass's word of live (cleared when the step
// begins) for a case that still needs an evaluation; a pass, and the finalize
// after it, read that one word first.  A pass that runs sees the same states as
// without the word, so the results do not depend on it.
__device__ __forceinline__ void mark_live(const CaseState &C, int32_t *live)
{
    if (live && C.state != RS_DONE && C.state != RS_FALLBACK) *live = 1;
}

// One workgroup per case.  Phases 0 (after the last stage) and 1 (before it, when
// the last stage evaluates the first residual): sums the stage entropy production
// of the b_i != 0 stages known so far in a fixed order, resets the solver state
// and sets the first evaluation point (the previous gamma, or that plus the
// learned increment); phase 0 also forms dH = dt sum_i b_i e_i.  Phase 2 (after
// such a last stage): adds the last stage's entropy production, forms dH and
// advances the solver with the evaluation the last stage made, as
// relax_finalize_kernel does after a residual pass.  Phases 0 and 2 raise *live
// for the first launched pass (live is null in phase 1).
__global__ void __launch_bounds__(PERRK_RED_THREADS)
relax_prepare_kernel(CaseState *cs, const int64_t *case_off, const double *ep, int64_t nelem,
                     RelaxParams rp, const float *mlp, int phase, const double *rx_partial,
                     const int32_t *case_chunk, const double *chunk_sums, int32_t *live)
{
    __shared__ float sx[8], sh1[32], sh2[32];
    const int c = blockIdx.x;
    const int64_t b = case_off[c], e = case_off[c + 1];
    const int k0 = case_chunk ? case_chunk[c] : 0, k1 = case_chunk ? case_chunk[c + 1] : 0;
    CaseState &C = cs[c];
    if (phase == 2) {
        double ej[PERRK_MAXB] = {};
        for (int j = rp.nb_pre; j < rp.nb; ++j) {
            double o[1];
            prep_sum<1>(ep + (size_t)j * nelem, 1, b, e, k0, k1, chunk_sums, j, o);
            ej[j] = o[0];
        }
        double S[4];
        prep_sum<4>(rx_partial, 4, b, e, k0, k1, chunk_sums, PERRK_MAXB, S);
        if (threadIdx.x != 0) return;
        double dH = 0.0;
        for (int j = 0; j < rp.nb; ++j) {
            if (j >= rp.nb_pre) C.e[j] = ej[j];
            dH += rp.bw[j] * C.e[j];
        }
        C.dH = C.dt * dH;
        if (C.state == RS_NEWTON) {
            relax_update(C, S, rp);
        } else if (C.state == RS_EVAL1) {  // no relaxation: the step's bookkeeping at gamma = 1
            const double off = (rp.anchor == 1) ? C.offset : 0.0;
            C.gamma_acc = 1.0;
            C.H_delta = S[0];
            C.r = S[0] - C.dH + off;
            C.state = RS_DONE;
        }  // (RS_BIS_INIT: no Newton budget; the residual passes open the bracket)
        mark_live(C, live);
        return;
    }
    const int nsum = phase == 0 ? rp.nb : rp.nb_pre;
    double ej[PERRK_MAXB] = {};
    for (int j = 0; j < nsum; ++j) {
        double o[1];
        prep_sum<1>(ep + (size_t)j * nelem, 1, b, e, k0, k1, chunk_sums, j, o);
        ej[j] = o[0];
    }
    // learned guess of the increment of the root, gamma*_n - gamma*_{n-1} (MLP
    // 8-32-32-1, tanh; the weights are followed by the feature mean[8], scale[8] and the
    // output scale and shift).  Features, formed in double precision from the history
    // of roots (ghist, see the step bookkeeping): the last two increments,
    // gamma*_{n-1} - 1, dt, and the entropy production of this step's b_i != 0 stages
    // before the last stage divided by the sum of their magnitudes (zero-padded to
    // four).  The first evaluation point is gamma*_{n-1} plus the prediction.
    const bool learned = rp.guess == 1 && mlp != nullptr && C.nsteps >= 3;
    const float *W1 = mlp, *b1 = W1 + 256, *W2 = b1 + 32, *b2 = W2 + 1024, *W3 = b2 + 32, *b3 = W3 + 32;
    const float *mean = b3 + 1, *scale = mean + 8, *oscale = scale + 8;
    if (learned) {
        if (threadIdx.x == 0) {
            double x[8];
            x[0] = C.ghist[0] - C.ghist[1];
            x[1] = C.ghist[1] - C.ghist[2];
            x[2] = C.ghist[0];
            x[3] = C.dt;
            double sabs = 0.0;
            for (int j = 0; j < rp.nb_pre; ++j) sabs += fabs(ej[j]);
            for (int j = 0; j < 4; ++j) x[4 + j] = (j < rp.nb_pre && sabs > 0.0) ? ej[j] / sabs : 0.0;
            for (int i = 0; i < 8; ++i) sx[i] = (float)((x[i] - (double)mean[i]) * (double)scale[i]);
        }
        __syncthreads();
        if (threadIdx.x < 32) {
            const int o = threadIdx.x;
            float s = b1[o];
            for (int i = 0; i < 8; ++i) s += W1[o * 8 + i] * sx[i];
            sh1[o] = tanhf(s);
        }
        __syncthreads();
        if (threadIdx.x < 32) {
            const int o = threadIdx.x;
            float s = b2[o];
            for (int i = 0; i < 32; ++i) s += W2[o * 32 + i] * sh1[i];
            sh2[o] = tanhf(s);
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double dH = 0.0;
    for (int j = 0; j < nsum; ++j) {
        C.e[j] = ej[j];
        dH += rp.bw[j] * ej[j];
    }
    if (phase == 0) C.dH = C.dt * dH;
    C.k = 0;
    C.iters = 0;
    C.passes = 0;
    C.flags = 0;
    C.bis_count = 0;
    C.widen = 0;
    C.r = 0.0;
    C.rp = 0.0;
    double g0 = C.gamma_prev;
    if (learned) {
        float y = b3[0];
        for (int i = 0; i < 32; ++i) y += W3[i] * sh2[i];
        const double pred = (double)y * (double)oscale[0] + (double)oscale[1];
        const double base = 1.0 + C.ghist[0];
        if (isfinite(pred) && fabs(pred) < 0.1 && base + pred > 0.0) g0 = base + pred;
    } else if (rp.guess == 2 && C.nsteps >= 2) {
        // linear extrapolation of the root history
        const double pred = C.ghist[0] - C.ghist[1];
        const double base = 1.0 + C.ghist[0];
        if (isfinite(pred) && fabs(pred) < 0.1 && base + pred > 0.0) g0 = base + pred;
    }
    C.gamma = g0;
    C.gamma_b = g0;
    C.H_delta = 0.0;
    C.state = rp.relax ? RS_NEWTON : RS_EVAL1;
    if (!rp.relax) C.gamma = 1.0;  // the step's bookkeeping evaluation is at gamma = 1
    if (rp.relax && rp.max_newton <= 0) {  // no Newton budget: open the bracket at once
        C.state = RS_BIS_INIT;
        C.flags |= PERRK_FLAG_BISECT;
        C.gamma = rp.bis_lo;
        C.gamma_b = rp.bis_hi;
    }
    C.gamma_acc = 1.0;
    mark_live(C, live);
}

template <int DIM, int SYS, bool FIRST>
__global__ void __launch_bounds__(256)
relax_pass_kernel(const double *U, const double *d, const ElemInfo *elem, const CaseState *cs,
                  double *partial, int64_t nelem, double gam, const int32_t *live_in)
{
    constexpr int NPE = Geo<DIM>::NPE, EPW = Geo<DIM>::EPW;
    // the block's elements are consecutive, so its cases are a contiguous range:
    // leave at once when every one of them is solved
    __shared__ int s_live;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t eb = (int64_t)blk * (blockDim.x >> 6) * EPW;
    int64_t ee = eb + (int64_t)(blockDim.x >> 6) * EPW - 1;
    if (ee >= nelem) ee = nelem - 1;
    if (!FIRST) {  // (in the first pass of a step every case is live)
        if (*live_in == 0) return;  // every case of the step is solved
        if (threadIdx.x == 0) {
            int live = 0;
            for (int c = elem[eb].case_id; c <= elem[ee].case_id; ++c) {
                const int st = cs[c].state;
                live |= (st != RS_DONE && st != RS_FALLBACK);
            }
            s_live = live;
        }
        __syncthreads();
        if (!s_live) return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t e0 = ((int64_t)blk * (blockDim.x >> 6) + wave) * EPW + lane / NPE;
    const bool valid = e0 < nelem;
    relax_element<DIM, SYS, true>(U, d, elem, cs, partial, nelem, gam, valid ? e0 : nelem - 1, lane % NPE, valid);
}

// Solver update of each case after a residual pass (live_in: the pass's word;
// live_out: the next pass's).
__global__ void __launch_bounds__(PERRK_RED_THREADS)
relax_finalize_kernel(CaseState *cs, const int64_t *case_off, const double *partial, RelaxParams rp,
                      const int32_t *live_in, int32_t *live_out)
{
    if (*live_in == 0) return;  // the pass did not run
    const int c = blockIdx.x;
    const int st = cs[c].state;
    if (st == RS_DONE || st == RS_FALLBACK) return;
    if (st != RS_EVAL1) {
        double S[4];
        case_sum<4>(partial, 4, case_off[c], case_off[c + 1], S);
        if (threadIdx.x == 0) relax_update(cs[c], S, rp);
    }
    if (threadIdx.x == 0) mark_live(cs[c], live_out);
}

// Runs the remaining residual evaluations of each case inside one workgroup
// (rarely needed: Newton usually converges within the launched passes), then
// the per-step bookkeeping.  Every evaluation uses the same per-element code and
// the same fixed-order sum as the launched passes.  A step that formed a
// non-physical or non-finite stage state (err[0] != 0) is rejected: the final
// update leaves u alone, so time, entropy offset and gamma history stay as
// they were too.
template <int DIM, int SYS>
__global__ void __launch_bounds__(PERRK_RED_THREADS)
relax_complete_kernel(const double *U, const double *d, const ElemInfo *elem, CaseState *cs,
                      const int64_t *case_off, double *partial, int64_t nelem, double gam,
                      RelaxParams rp, const int32_t *err)
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
            relax_element<DIM, SYS>(U, d, elem, cs, partial, nelem, gam, valid ? el : e - 1, lane % NPE,
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
        if (err[0] != 0) return;
        C.t += C.gamma_acc * C.dt;
        C.offset += C.H_delta;
        // history of the learned guess: the root itself rather than the accepted point.
        // An evaluation accepted by Newton gave r and r' there, and one more Newton step
        // locates the root far inside the acceptance band |r| <= tol_r, where the
        // accepted points scatter by about tol_r / |r'| from step to step
        double groot = C.gamma_acc;
        if (C.flags == 0 && C.passes > 0 && isfinite(C.r) && isfinite(C.rp) && C.rp != 0.0) {
            const double corr = C.r / C.rp;
            if (fabs(corr) < 1e-6) groot -= corr;
        }
        C.ghist[2] = C.ghist[1];
        C.ghist[1] = C.ghist[0];
        C.ghist[0] = groot - 1.0;
        C.gamma_prev = C.gamma_acc;
        C.nsteps += 1;
    }
}

// U <- U + gamma dt d, two doubles per thread; skipped entirely after an error
// of this step (err[0]), which is then added to the errors not yet reported
// (err[1]).
template <int DIM, int SYS>
__global__ void __launch_bounds__(256)
final_update_kernel(double *U, const double *d, const ElemInfo *elem, const CaseState *cs,
                    int32_t *err, int64_t nelem)
{
    constexpr int NPE = Sys<DIM, SYS>::NPE, V = Sys<DIM, SYS>::V;
    const int32_t e_step = err[0];
    if (e_step != 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) err[1] |= e_step;
        return;
    }
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

template <int DIM, int SYS>
__global__ void __launch_bounds__(256)
entropy_elem_kernel(const double *U, const ElemInfo *elem, double *partial, int64_t nelem, double gam,
                    int32_t *err)
{
    constexpr int NPE = Sys<DIM, SYS>::NPE, V = Sys<DIM, SYS>::V, EPW = Sys<DIM, SYS>::EPW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t e0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * EPW + lane / NPE;
    const bool valid = e0 < nelem;
    const int64_t e = valid ? e0 : nelem - 1;
    const int node = lane % NPE;
    double u[V];
#pragma unroll
    for (int v = 0; v < V; ++v) u[v] = U[((size_t)v * nelem + e) * NPE + node];
    double s = node_weight<DIM>(node) * (SYS == 1 ? mhd_entropy_density(u, gam) : entropy_density<DIM>(u, gam));
    int bad = 0;
    if constexpr (SYS == 1) {
        PrimM P;
        make_prim_mhd(u, gam - 1.0, P, bad);
    } else {
        Prim<double, DIM> P;
        make_prim<double, DIM>(u, gam - 1.0, P, bad);
    }
#pragma unroll
    for (int off = NPE / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (valid && node == 0) partial[e] = elem[e].jac * s;
    if (valid && node == 0 && !isfinite(s)) bad |= 2;
    if (valid && bad) atomicOr(err, (bad & 1) ? 1 : bad);
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

__global__ void clear_err_kernel(int32_t *err, int n)
{
    if ((int)threadIdx.x < n) err[threadIdx.x] = 0;
}

__global__ void clear_step_kernel(int32_t *err_step, int32_t *live, int n_live)
{
    if (threadIdx.x == 0) *err_step = 0;
    if ((int)threadIdx.x < n_live) live[threadIdx.x] = 0;
}

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

template <int DIM, typename T, typename KT, int FLUX, int KIND, bool ONE_DIR>
hipError_t launch_stage_s(const StageArgs &a, const double *coef, LaunchCfg cfg, hipStream_t s)
{
    constexpr int EPW = SG<DIM>::EPW, SLOT = SL<DIM, T, SplitDirs<DIM, FLUX, ONE_DIR>::ON>::SLOT;
    const int wpb = cfg.epb_mult;
    const int epb = wpb * EPW;
    if (a.n_active <= 0) return hipSuccess;
    const int blocks = (a.n_active + epb - 1) / epb;
    // single precision: the element slots, then one gather table per wavefront
    const size_t lds = ((size_t)epb * SLOT + (sizeof(T) == 4 ? (size_t)wpb * GTAB_WORDS : 0)) * sizeof(T);
    hipLaunchKernelGGL((stage_kernel<DIM, T, KT, FLUX, KIND, ONE_DIR>), dim3(blocks), dim3(64 * wpb), lds, s, a,
                       coef);
    return hipGetLastError();
}

template <int DIM, typename T, typename KT, int FLUX, int KIND>
hipError_t launch_stage_t(const StageArgs &a, const double *coef, LaunchCfg cfg, hipStream_t s)
{
    if constexpr (SplitDirs<DIM, FLUX, true>::ON) {
        if (cfg.one_dir) return launch_stage_s<DIM, T, KT, FLUX, KIND, true>(a, coef, cfg, s);
    }
    return launch_stage_s<DIM, T, KT, FLUX, KIND, false>(a, coef, cfg, s);
}

template <int DIM, typename T, typename KT, int FLUX>
hipError_t launch_stage_k(int kind, const StageArgs &a, const double *coef, LaunchCfg cfg, hipStream_t s)
{
    if (kind == SK_FIRST) return launch_stage_t<DIM, T, KT, FLUX, SK_FIRST>(a, coef, cfg, s);
    if (kind == SK_MID) return launch_stage_t<DIM, T, KT, FLUX, SK_MID>(a, coef, cfg, s);
    return launch_stage_t<DIM, T, KT, FLUX, SK_LAST>(a, coef, cfg, s);
}

// variant: 0 = double flux / double storage, 1 = float flux / float storage,
// 2 = double flux / float storage (stages with b_i != 0 in mixed precision)
template <int DIM, int FLUX>
hipError_t launch_stage_v(int variant, int kind, const StageArgs &a, const double *coef, LaunchCfg cfg,
                          hipStream_t s)
{
    if (variant == 1) return launch_stage_k<DIM, float, float, FLUX>(kind, a, coef, cfg, s);
    if (variant == 2) return launch_stage_k<DIM, double, float, FLUX>(kind, a, coef, cfg, s);
    return launch_stage_k<DIM, double, double, FLUX>(kind, a, coef, cfg, s);
}

template <int DIM>
hipError_t launch_stage_d(int variant, int flux, int kind, const StageArgs &a, const double *coef,
                          LaunchCfg cfg, hipStream_t s)
{
    if (flux || a.volume) return launch_stage_v<DIM, 1>(variant, kind, a, coef, cfg, s);
    return launch_stage_v<DIM, 0>(variant, kind, a, coef, cfg, s);
}

template <int KIND>
hipError_t launch_mhd_stage_t(const StageArgs &a, const double *coef, LaunchCfg cfg, hipStream_t s)
{
    const int wpb = cfg.epb_mult;
    const int epb = wpb * 4;
    if (a.n_active <= 0) return hipSuccess;
    const int blocks = (a.n_active + epb - 1) / epb;
    if (cfg.one_dir) {
        const size_t lds = (size_t)epb * mhd_slot<true>() * sizeof(double);
        hipLaunchKernelGGL((mhd_stage_kernel<KIND, true>), dim3(blocks), dim3(64 * wpb), lds, s, a, coef);
    } else {
        const size_t lds = (size_t)epb * mhd_slot<false>() * sizeof(double);
        hipLaunchKernelGGL((mhd_stage_kernel<KIND, false>), dim3(blocks), dim3(64 * wpb), lds, s, a, coef);
    }
    return hipGetLastError();
}

// Navier-Stokes stage: the gradient pass over every element (its own stage
// state, the neighbours' at the faces), then the stage kernel over the stage's
// active elements.
template <int KIND>
hipError_t launch_ns_stage_t(const StageArgs &a, const double *coef, LaunchCfg cfg, hipStream_t s)
{
    const int wpb = cfg.epb_mult;
    const int epb = wpb * 4;
    if (a.n_all > 0) {
        StageArgs g = a;
        g.active = a.active_all;
        g.n_active = a.n_all;
        const int blocks = (g.n_active + epb - 1) / epb;
        hipLaunchKernelGGL((ns_grad_kernel<KIND>), dim3(blocks), dim3(64 * wpb),
                           (size_t)epb * NS_GRAD_SLOT * sizeof(double), s, g, coef);
    }
    if (a.n_active <= 0) return hipGetLastError();
    const int blocks = (a.n_active + epb - 1) / epb;
    hipLaunchKernelGGL((ns_stage_kernel<KIND>), dim3(blocks), dim3(64 * wpb), (size_t)epb * NS_SLOT * sizeof(double),
                       s, a, coef);
    return hipGetLastError();
}

}  // namespace

size_t stage_lds_bytes(int dim, int variant, int wpb, int sys, bool one_dir)
{
    if (sys == 1) return (size_t)wpb * 4 * (one_dir ? mhd_slot<true>() : mhd_slot<false>()) * sizeof(double);
    if (sys == 2) return (size_t)wpb * 4 * NS_SLOT * sizeof(double);
    const bool ec = one_dir;  // (quadrilaterals with the EC fluxes only)
    if (variant == 1) {  // element slots and the wavefronts' gather tables
        if (dim == 2)
            return (size_t)wpb * (SG<2>::EPW * (ec ? SL<2, float, true>::SLOT : SL<2, float>::SLOT) + GTAB_WORDS) *
                   sizeof(float);
        return (size_t)wpb * (SG<3>::EPW * (ec ? SL<3, float, true>::SLOT : SL<3, float>::SLOT) + GTAB_WORDS) *
               sizeof(float);
    }
    if (dim == 2) return (size_t)wpb * SG<2>::EPW * (ec ? SL<2, double, true>::SLOT : SL<2, double>::SLOT) * sizeof(double);
    return (size_t)wpb * SG<3>::EPW * (ec ? SL<3, double, true>::SLOT : SL<3, double>::SLOT) * sizeof(double);
}

hipError_t launch_stage(int dim, int variant, int flux, int kind, const StageArgs &a, const double *coef,
                        LaunchCfg cfg, hipStream_t s)
{
    if (cfg.epb_mult < 1 || cfg.epb_mult > PERRK_MAX_WPB) return hipErrorInvalidValue;
    if (a.viscous) {  // Navier-Stokes-Fourier: 2D, double precision
        if (dim != 2 || variant != 0 || a.sys != 0) return hipErrorInvalidValue;
        if (kind == SK_FIRST) return launch_ns_stage_t<SK_FIRST>(a, coef, cfg, s);
        if (kind == SK_MID) return launch_ns_stage_t<SK_MID>(a, coef, cfg, s);
        return launch_ns_stage_t<SK_LAST>(a, coef, cfg, s);
    }
    if (a.sys == 1) {  // ideal GLM-MHD: 2D, double precision
        if (dim != 2 || variant != 0) return hipErrorInvalidValue;
        if (kind == SK_FIRST) return launch_mhd_stage_t<SK_FIRST>(a, coef, cfg, s);
        if (kind == SK_MID) return launch_mhd_stage_t<SK_MID>(a, coef, cfg, s);
        return launch_mhd_stage_t<SK_LAST>(a, coef, cfg, s);
    }
    if (dim == 2) return launch_stage_d<2>(variant, flux, kind, a, coef, cfg, s);
    return launch_stage_d<3>(variant, flux, kind, a, coef, cfg, s);
}

hipError_t launch_relax_prepare(CaseState *cs, const int64_t *case_off, int n_cases, const double *ep,
                                int64_t nelem, RelaxParams rp, const float *mlp, int phase,
                                const double *rx_partial, const PrepChunks &ch, int32_t *live, hipStream_t s)
{
    if (ch.n_chunks > 0) {
        hipLaunchKernelGGL(prepare_chunks_kernel, dim3(ch.n_chunks), dim3(PERRK_RED_THREADS), 0, s, ch.range, ep,
                           nelem, rp, phase, rx_partial, ch.sums);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(relax_prepare_kernel, dim3(n_cases), dim3(PERRK_RED_THREADS), 0, s, cs, case_off,
                       ep, nelem, rp, mlp, phase, rx_partial, ch.n_chunks > 0 ? ch.case_chunk : nullptr,
                       ch.sums, phase == 1 ? nullptr : live);
    return hipGetLastError();
}

hipError_t launch_relax_pass(int dim, int sys, const double *U, const double *d, const ElemInfo *elem,
                             const CaseState *cs, double *partial, int64_t nelem, double gam, bool first,
                             const int32_t *live, hipStream_t s)
{
    const int epw = dim == 2 ? 4 : 1;
    const int64_t waves = (nelem + epw - 1) / epw;
    const int64_t blocks = (waves + 3) / 4;
#define PERRK_PASS(D, SY)                                                                                   \
    do {                                                                                                   \
        if (first)                                                                                         \
            hipLaunchKernelGGL((relax_pass_kernel<D, SY, true>), dim3((unsigned)blocks), dim3(256), 0, s, U, d, \
                               elem, cs, partial, nelem, gam, live);                                       \
        else                                                                                               \
            hipLaunchKernelGGL((relax_pass_kernel<D, SY, false>), dim3((unsigned)blocks), dim3(256), 0, s, U, d, \
                               elem, cs, partial, nelem, gam, live);                                       \
    } while (0)
    if (sys == 1) PERRK_PASS(2, 1);
    else if (dim == 2) PERRK_PASS(2, 0);
    else PERRK_PASS(3, 0);
#undef PERRK_PASS
    return hipGetLastError();
}

hipError_t launch_relax_finalize(CaseState *cs, const int64_t *case_off, int n_cases, const double *partial,
                                 RelaxParams rp, const int32_t *live_in, int32_t *live_out, hipStream_t s)
{
    hipLaunchKernelGGL(relax_finalize_kernel, dim3(n_cases), dim3(PERRK_RED_THREADS), 0, s, cs, case_off,
                       partial, rp, live_in, live_out);
    return hipGetLastError();
}

hipError_t launch_relax_complete(int dim, int sys, const double *U, const double *d, const ElemInfo *elem,
                                 CaseState *cs, const int64_t *case_off, int n_cases, double *partial,
                                 int64_t nelem, double gam, RelaxParams rp, const int32_t *err, hipStream_t s)
{
    if (sys == 1)
        hipLaunchKernelGGL((relax_complete_kernel<2, 1>), dim3(n_cases), dim3(PERRK_RED_THREADS), 0, s, U, d,
                           elem, cs, case_off, partial, nelem, gam, rp, err);
    else if (dim == 2)
        hipLaunchKernelGGL((relax_complete_kernel<2, 0>), dim3(n_cases), dim3(PERRK_RED_THREADS), 0, s, U, d,
                           elem, cs, case_off, partial, nelem, gam, rp, err);
    else
        hipLaunchKernelGGL((relax_complete_kernel<3, 0>), dim3(n_cases), dim3(PERRK_RED_THREADS), 0, s, U, d,
                           elem, cs, case_off, partial, nelem, gam, rp, err);
    return hipGetLastError();
}

hipError_t launch_final_update(int dim, int sys, double *U, const double *d, const ElemInfo *elem,
                               const CaseState *cs, int32_t *err, int64_t nelem, hipStream_t s)
{
    const int npe = dim == 2 ? 16 : 64;
    const int64_t n2 = (int64_t)(sys == 1 ? MHD_V : dim + 2) * nelem * npe / 2;
    int64_t blocks = (n2 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (sys == 1)
        hipLaunchKernelGGL((final_update_kernel<2, 1>), dim3((unsigned)blocks), dim3(256), 0, s, U, d, elem, cs,
                           err, nelem);
    else if (dim == 2)
        hipLaunchKernelGGL((final_update_kernel<2, 0>), dim3((unsigned)blocks), dim3(256), 0, s, U, d, elem, cs,
                           err, nelem);
    else
        hipLaunchKernelGGL((final_update_kernel<3, 0>), dim3((unsigned)blocks), dim3(256), 0, s, U, d, elem, cs,
                           err, nelem);
    return hipGetLastError();
}

hipError_t launch_entropy(int dim, int sys, const double *U, const ElemInfo *elem, double *partial, double *H_out,
                          const int64_t *case_off, int n_cases, int64_t nelem, double gam, int32_t *err,
                          hipStream_t s)
{
    const int epw = dim == 2 ? 4 : 1;
    const int64_t blocks = ((nelem + epw - 1) / epw + 3) / 4;
    if (sys == 1)
        hipLaunchKernelGGL((entropy_elem_kernel<2, 1>), dim3((unsigned)blocks), dim3(256), 0, s, U, elem, partial,
                           nelem, gam, err);
    else if (dim == 2)
        hipLaunchKernelGGL((entropy_elem_kernel<2, 0>), dim3((unsigned)blocks), dim3(256), 0, s, U, elem, partial,
                           nelem, gam, err);
    else
        hipLaunchKernelGGL((entropy_elem_kernel<3, 0>), dim3((unsigned)blocks), dim3(256), 0, s, U, elem, partial,
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

hipError_t launch_clear_err(int32_t *err, int n, hipStream_t s)
{
    hipLaunchKernelGGL(clear_err_kernel, dim3(1), dim3(64), 0, s, err, n);
    return hipGetLastError();
}

hipError_t launch_clear_step(int32_t *err_step, int32_t *live, int n_live, hipStream_t s)
{
    if (n_live < 0 || n_live > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(clear_step_kernel, dim3(1), dim3(64), 0, s, err_step, live, n_live);
    return hipGetLastError();
}
