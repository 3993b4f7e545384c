/*
 * perrk_oracle.c -- plain FP64 CPU oracle for one P-ERRK step on a periodic
 * Cartesian DGSEM (degree 3) discretisation of the compressible Euler
 * equations.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The product path
 * (the HIP library behind include/perrk.h) shares no code with it.
 *
 * Everything is written as slow, obvious loops in double precision, in the
 * order of the paper:
 *   - Sec. 2.1: semidiscretisation U' = F(U) by DGSEM on LGL nodes;
 *     entropy-conservative flux differencing in the volume, entropy-conservative
 *     or entropy-stable surface fluxes (the paper cites these; their formulas are
 *     restated here from the published mathematics: Ranocha's EC/KEP flux, the
 *     HLL two-wave solver with Davis speeds, and the dissipative fluxes of the
 *     validation and application runs of Sec. 4.2, 4.3 and 5: local
 *     Lax-Friedrichs, HLLE, HLLC); the standard weak-form volume integral of
 *     the linear-invariant test of Sec. 4.2 as an alternative volume term.
 *   - Sec. 2.2: partitioned RK in Butcher form (PartitionedRKSystem), the
 *     archetype tableaux of Appendix A, the active-stage rule and the cheap
 *     update of inactive partitions.
 *   - Sec. 2.3: entropy s(u) = -rho log(p / rho^gamma) (EntropyMathematical).
 *   - Sec. 4.1.1 and 4.3.3: ideal GLM-MHD as a second system (nine variables,
 *     the same entropy with the MHD pressure, an EC two-point flux, the Powell
 *     and GLM non-conservative terms, LLF and central surface fluxes).
 *   - Sec. 2.4 / 3: relaxed update U_{n+1} = U_n + gamma dt d, entropy change
 *     Delta H from the stage entropy production (EntropyChangeDefinition,
 *     its rearranged node-wise form), relaxation residual r(gamma) and its
 *     derivative (RelaxationEquation), Newton with unit step, bisection.
 *
 * Layout at the interface: structure of arrays U[v][elem][node], node fastest,
 * node = i + 4 j + 16 k (x index fastest), elem = ix + nx (iy + ny iz).
 * Conserved variables per node: rho, rho v_1..rho v_dim, rho e.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_N 4            /* LGL nodes per direction */
#define OR_MAXS 64        /* maximum number of stages */
#define OR_MAXR 32        /* maximum number of levels */
#define OR_MAXV 9         /* maximum number of conserved variables per node */

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_ENONPHYS = -4, OR_ENONFINITE = -5 };
enum { OR_FLAG_BISECT = 1, OR_FLAG_FALLBACK = 2, OR_FLAG_TRIVIAL = 4 };

typedef struct {
    int dim;              /* 2 or 3 */
    int n[3];             /* elements per direction; n[2] = 1 in 2D */
    const double *faces;  /* face coordinates, direction 0 then 1 (then 2): n[d]+1 each */
    double gam;           /* ratio of specific heats */
    int surface_flux;     /* 0: Ranocha EC flux, 1: HLL (Davis speeds), 2: local Lax-Friedrichs,
                             3: HLLE (Einfeldt speeds), 4: HLLC (Davis speeds) */
    int volume_integral;  /* 0: flux differencing with the EC flux, 1: standard weak form */
    int physics;          /* 0: compressible Euler (V = dim + 2), 1: ideal GLM-MHD (V = 9) */
    double c_h;           /* GLM-MHD: divergence-cleaning speed */
    int viscous;          /* Euler only: 1 adds the Navier-Stokes-Fourier terms (BR1), 2D */
    double mu, prandtl;   /* dynamic viscosity, Prandtl number (kappa = gamma mu / ((gamma-1) Pr)) */
    int bc_x;             /* 0: periodic in x; 1: the viscous-shock boundaries at both x ends */
    double time;          /* time of the state the boundary values are taken at (set per stage) */
} or_mesh;

typedef struct {
    int order;            /* 2, 3 or 4 (informational) */
    int S;                /* number of stages */
    int R;                /* number of levels */
    const int *E;         /* [R] stage evaluations of each level */
    const double *c;      /* [S] abscissae, shared by all levels */
    const double *b;      /* [S] weights, shared by all levels (Conservation) */
    const double *a_sub;  /* [R][S] a^{(r)}_{i,i-1}; a^{(r)}_{i,1} = c_i - a^{(r)}_{i,i-1} */
} or_tableau;

typedef struct {
    int relax;            /* 0: plain P-ERK step, gamma = 1 */
    int max_newton;
    double tol_r;         /* accept gamma only when |r(gamma)| <= tol_r */
    double tol_step;      /* a Newton step below this ends the Newton loop */
    int anchor;           /* 0: H(U_{n+1}) = H(U_n) + gamma dH ; 1: ... = H0 + gamma dH */
    double H0;
    double bis_lo, bis_hi;
    int max_bisect;
    double gamma0;        /* initial guess of the Newton iteration */
    double t0;            /* time of U_n (for time-dependent boundary values) */
} or_relax;

typedef struct {
    double gamma, r, dH, H_old, H_new;
    int passes, newton_iters, flags, pad;
    double e[OR_MAXS];    /* stage entropy production <W(U_{n,i}), K_i> for b_i != 0 */
} or_info;

/* ------------------------------------------------------------------------ */
/* LGL nodes, weights, derivative matrix, split-form matrix (degree 3)       */
/* ------------------------------------------------------------------------ */

/* Nodes: roots of (1 - x^2) P_3'(x); weights 2/(N(N+1) P_3(x)^2), N = 3.
 * D_ij = l_j'(xi_i) from the barycentric form of the Lagrange basis.
 * Dsplit = 2 D - W^{-1} B, B = diag(-1, 0, 0, 1): the flux-differencing form
 * of the DGSEM volume term (its diagonal vanishes). */
void or_lgl(double *xi, double *q, double *D, double *Dsplit)
{
    const double s = 1.0 / sqrt(5.0);
    double x[OR_N] = { -1.0, -s, s, 1.0 };
    double w[OR_N] = { 1.0 / 6.0, 5.0 / 6.0, 5.0 / 6.0, 1.0 / 6.0 };
    double lam[OR_N];
    for (int j = 0; j < OR_N; ++j) {
        double p = 1.0;
        for (int k = 0; k < OR_N; ++k)
            if (k != j) p *= (x[j] - x[k]);
        lam[j] = 1.0 / p;
    }
    for (int i = 0; i < OR_N; ++i) {
        double diag = 0.0;
        for (int j = 0; j < OR_N; ++j) {
            if (j == i) continue;
            double dij = (lam[j] / lam[i]) / (x[i] - x[j]);
            D[i * OR_N + j] = dij;
            diag -= dij;
        }
        D[i * OR_N + i] = diag;
    }
    for (int i = 0; i < OR_N; ++i) {
        xi[i] = x[i];
        q[i] = w[i];
        for (int j = 0; j < OR_N; ++j) {
            double bij = 0.0;
            if (i == j && i == 0) bij = -1.0;
            if (i == j && i == OR_N - 1) bij = 1.0;
            Dsplit[i * OR_N + j] = 2.0 * D[i * OR_N + j] - bij / w[i];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Thermodynamics                                                            */
/* ------------------------------------------------------------------------ */

/* Logarithmic mean (a - b) / (log a - log b).  With z = (a-b)/(a+b),
 * log(a/b) = 2 (z + z^3/3 + z^5/5 + z^7/7 + ...), hence for small z the mean
 * equals (a+b) / (2 + 2z^2/3 + 2z^4/5 + 2z^6/7 + ...), truncated after z^6
 * (omitted term < z^8 / 9 < 1.2e-17 relative for z^2 < 1e-4).  Otherwise the
 * logarithm of the ratio is taken as log1p((a-b)/b), which avoids the
 * cancellation of log a - log b for nearby arguments. */
double or_logmean(double a, double b)
{
    double z = (a - b) / (a + b);
    double z2 = z * z;
    if (z2 < 1.0e-4)
        return (a + b) / (2.0 + z2 * (2.0 / 3.0 + z2 * (2.0 / 5.0 + z2 * (2.0 / 7.0))));
    return (a - b) / log1p((a - b) / b);
}

/* Primitive variables of a node state; returns 0, ENONPHYS or ENONFINITE. */
static int or_prim(int dim, const double *u, double gam, double *rho, double *v, double *p)
{
    for (int k = 0; k < dim + 2; ++k)
        if (!isfinite(u[k])) return OR_ENONFINITE;
    *rho = u[0];
    if (!(*rho > 0.0)) return OR_ENONPHYS;
    double kin = 0.0;
    for (int d = 0; d < dim; ++d) {
        v[d] = u[1 + d] / u[0];
        kin += 0.5 * u[1 + d] * v[d];
    }
    *p = (gam - 1.0) * (u[dim + 1] - kin);
    if (!(*p > 0.0)) return OR_ENONPHYS;
    return OR_OK;
}

/* Physical Euler flux in direction dir. */
void or_flux_phys(int dim, int dir, const double *u, double gam, double *f)
{
    double rho, v[3], p;
    or_prim(dim, u, gam, &rho, v, &p);
    double vn = v[dir];
    f[0] = u[0] * vn;
    for (int d = 0; d < dim; ++d) f[1 + d] = u[1 + d] * vn + (d == dir ? p : 0.0);
    f[dim + 1] = (u[dim + 1] + p) * vn;
}

/* Ranocha's entropy-conservative, kinetic-energy-preserving two-point flux
 * (the EC volume and surface flux of Sec. 4.1).  With arithmetic means {.}
 * and logarithmic means {.}_log:
 *   f_rho = {rho}_log {v_n}
 *   f_m   = f_rho {v} + {p} n
 *   f_E   = f_rho ( v_L . v_R / 2 + 1 / ((gamma-1) {rho/p}_log) )
 *           + (p_L v_n,R + p_R v_n,L) / 2                                   */
void or_flux_ec(int dim, int dir, const double *uL, const double *uR, double gam, double *f)
{
    double rl, rr, vl[3], vr[3], pl, pr;
    or_prim(dim, uL, gam, &rl, vl, &pl);
    or_prim(dim, uR, gam, &rr, vr, &pr);
    double rho_log = or_logmean(rl, rr);
    double beta_log = or_logmean(rl / pl, rr / pr);
    double vn_avg = 0.5 * (vl[dir] + vr[dir]);
    double p_avg = 0.5 * (pl + pr);
    double vv = 0.0;
    for (int d = 0; d < dim; ++d) vv += vl[d] * vr[d];
    double frho = rho_log * vn_avg;
    f[0] = frho;
    for (int d = 0; d < dim; ++d) f[1 + d] = frho * 0.5 * (vl[d] + vr[d]) + (d == dir ? p_avg : 0.0);
    f[dim + 1] = frho * (0.5 * vv + 1.0 / ((gam - 1.0) * beta_log)) + 0.5 * (pl * vr[dir] + pr * vl[dir]);
}

/* HLL two-wave flux with Davis wave-speed estimates
 *   lmin = min(vn_L - c_L, vn_R - c_R),  lmax = max(vn_L + c_L, vn_R + c_R). */
void or_flux_hll(int dim, int dir, const double *uL, const double *uR, double gam, double *f)
{
    double rl, rr, vl[3], vr[3], pl, pr;
    or_prim(dim, uL, gam, &rl, vl, &pl);
    or_prim(dim, uR, gam, &rr, vr, &pr);
    double cl = sqrt(gam * pl / rl), cr = sqrt(gam * pr / rr);
    double lmin = fmin(vl[dir] - cl, vr[dir] - cr);
    double lmax = fmax(vl[dir] + cl, vr[dir] + cr);
    double fl[5], fr[5];
    or_flux_phys(dim, dir, uL, gam, fl);
    or_flux_phys(dim, dir, uR, gam, fr);
    int V = dim + 2;
    if (lmin >= 0.0) {
        for (int k = 0; k < V; ++k) f[k] = fl[k];
    } else if (lmax <= 0.0) {
        for (int k = 0; k < V; ++k) f[k] = fr[k];
    } else {
        for (int k = 0; k < V; ++k)
            f[k] = (lmax * fl[k] - lmin * fr[k] + lmin * lmax * (uR[k] - uL[k])) / (lmax - lmin);
    }
}

/* Local Lax-Friedrichs (Rusanov) flux
 *   f = (f(u_L) + f(u_R)) / 2 - lambda (u_R - u_L) / 2,
 *   lambda = max(|vn_L| + c_L, |vn_R| + c_R). */
void or_flux_llf(int dim, int dir, const double *uL, const double *uR, double gam, double *f)
{
    double rl, rr, vl[3], vr[3], pl, pr;
    or_prim(dim, uL, gam, &rl, vl, &pl);
    or_prim(dim, uR, gam, &rr, vr, &pr);
    double cl = sqrt(gam * pl / rl), cr = sqrt(gam * pr / rr);
    double lam = fmax(fabs(vl[dir]) + cl, fabs(vr[dir]) + cr);
    double fl[5], fr[5];
    or_flux_phys(dim, dir, uL, gam, fl);
    or_flux_phys(dim, dir, uR, gam, fr);
    for (int k = 0; k < dim + 2; ++k) f[k] = 0.5 * (fl[k] + fr[k]) - 0.5 * lam * (uR[k] - uL[k]);
}

/* HLL flux with Einfeldt's wave speeds (HLLE): Roe averages with weights
 * sqrt(rho) give vn~ and c~^2 = (gamma-1) (H~ - |v~|^2 / 2), H = (E + p) / rho;
 *   lmin = min(vn_L - c_L, vn~ - c~),  lmax = max(vn_R + c_R, vn~ + c~),
 * then the two-wave formula (upwind when all speeds have one sign). */
void or_flux_hlle(int dim, int dir, const double *uL, const double *uR, double gam, double *f)
{
    double rl, rr, vl[3], vr[3], pl, pr;
    or_prim(dim, uL, gam, &rl, vl, &pl);
    or_prim(dim, uR, gam, &rr, vr, &pr);
    double cl = sqrt(gam * pl / rl), cr = sqrt(gam * pr / rr);
    double sl = sqrt(rl), sr = sqrt(rr);
    double hl = (uL[dim + 1] + pl) / rl, hr = (uR[dim + 1] + pr) / rr;
    double vt[3], v2 = 0.0;
    for (int d = 0; d < dim; ++d) {
        vt[d] = (sl * vl[d] + sr * vr[d]) / (sl + sr);
        v2 += vt[d] * vt[d];
    }
    double ht = (sl * hl + sr * hr) / (sl + sr);
    double ct = sqrt((gam - 1.0) * (ht - 0.5 * v2));
    double lmin = fmin(vl[dir] - cl, vt[dir] - ct);
    double lmax = fmax(vr[dir] + cr, vt[dir] + ct);
    double fl[5], fr[5];
    or_flux_phys(dim, dir, uL, gam, fl);
    or_flux_phys(dim, dir, uR, gam, fr);
    int V = dim + 2;
    if (lmin >= 0.0) {
        for (int k = 0; k < V; ++k) f[k] = fl[k];
    } else if (lmax <= 0.0) {
        for (int k = 0; k < V; ++k) f[k] = fr[k];
    } else {
        for (int k = 0; k < V; ++k)
            f[k] = (lmax * fl[k] - lmin * fr[k] + lmin * lmax * (uR[k] - uL[k])) / (lmax - lmin);
    }
}

/* HLLC flux (three waves; Toro's formulation) with the Davis wave speeds of
 * or_flux_hll.  Contact speed
 *   s* = (p_R - p_L + rho_L vn_L (sL - vn_L) - rho_R vn_R (sR - vn_R))
 *        / (rho_L (sL - vn_L) - rho_R (sR - vn_R)),
 * star state of side K: rho_K (sK - vn_K) / (sK - s*) times
 *   (1, v_K with its normal component replaced by s*,
 *    E_K / rho_K + (s* - vn_K) (s* + p_K / (rho_K (sK - vn_K)))),
 * flux f_K + sK (u*_K - u_K) on the side of the contact that holds x = 0. */
void or_flux_hllc(int dim, int dir, const double *uL, const double *uR, double gam, double *f)
{
    double rl, rr, vl[3], vr[3], pl, pr;
    or_prim(dim, uL, gam, &rl, vl, &pl);
    or_prim(dim, uR, gam, &rr, vr, &pr);
    double cl = sqrt(gam * pl / rl), cr = sqrt(gam * pr / rr);
    double sL = fmin(vl[dir] - cl, vr[dir] - cr);
    double sR = fmax(vl[dir] + cl, vr[dir] + cr);
    double fl[5], fr[5];
    or_flux_phys(dim, dir, uL, gam, fl);
    or_flux_phys(dim, dir, uR, gam, fr);
    int V = dim + 2;
    if (sL >= 0.0) {
        for (int k = 0; k < V; ++k) f[k] = fl[k];
        return;
    }
    if (sR <= 0.0) {
        for (int k = 0; k < V; ++k) f[k] = fr[k];
        return;
    }
    double ml = rl * (sL - vl[dir]), mr = rr * (sR - vr[dir]);
    double ss = (pr - pl + ml * vl[dir] - mr * vr[dir]) / (ml - mr);
    const int left = ss >= 0.0;
    const double *u = left ? uL : uR, *fk = left ? fl : fr, *vk = left ? vl : vr;
    double rk = left ? rl : rr, pk = left ? pl : pr, sk = left ? sL : sR, mk = left ? ml : mr;
    double fac = mk / (sk - ss);
    double us[5];
    us[0] = fac;
    for (int d = 0; d < dim; ++d) us[1 + d] = fac * (d == dir ? ss : vk[d]);
    us[dim + 1] = fac * (u[dim + 1] / rk + (ss - vk[dir]) * (ss + pk / mk));
    for (int k = 0; k < V; ++k) f[k] = fk[k] + sk * (us[k] - u[k]);
}

/* The surface flux selected for the mesh. */
static void or_surface_flux(const or_mesh *m, int dir, const double *uL, const double *uR, double *f)
{
    switch (m->surface_flux) {
    case 1: or_flux_hll(m->dim, dir, uL, uR, m->gam, f); break;
    case 2: or_flux_llf(m->dim, dir, uL, uR, m->gam, f); break;
    case 3: or_flux_hlle(m->dim, dir, uL, uR, m->gam, f); break;
    case 4: or_flux_hllc(m->dim, dir, uL, uR, m->gam, f); break;
    default: or_flux_ec(m->dim, dir, uL, uR, m->gam, f);
    }
}

/* Mathematical entropy s(u) = -rho log(p / rho^gamma) (Sec. 2.3). */
double or_entropy(int dim, const double *u, double gam)
{
    double rho, v[3], p;
    or_prim(dim, u, gam, &rho, v, &p);
    return -rho * (log(p) - gam * log(rho));
}

/* Entropy variables w = ds/du for the entropy above:
 *   w_rho = gamma - log(p rho^-gamma) - (gamma-1) rho |v|^2 / (2p)
 *   w_m   = (gamma-1) rho v / p
 *   w_E   = -(gamma-1) rho / p                                               */
void or_entropy_vars(int dim, const double *u, double gam, double *w)
{
    double rho, v[3], p;
    or_prim(dim, u, gam, &rho, v, &p);
    double v2 = 0.0;
    for (int d = 0; d < dim; ++d) v2 += v[d] * v[d];
    double rp = rho / p;
    w[0] = gam - (log(p) - gam * log(rho)) - 0.5 * (gam - 1.0) * rp * v2;
    for (int d = 0; d < dim; ++d) w[1 + d] = (gam - 1.0) * rp * v[d];
    w[dim + 1] = -(gam - 1.0) * rp;
}

/* s(u + du) - s(u) without cancellation.  With rho' = rho + drho and
 *   dp = (gamma-1) [ dE - (m.dm + |dm|^2/2) / rho' + drho |m|^2 / (2 rho rho') ]
 * (exactly p(u+du) - p(u)), one has
 *   s(u+du) - s(u) = -drho (log p' - gamma log rho')
 *                    - rho [ log1p(dp/p) - gamma log1p(drho/rho) ].          */
double or_entropy_diff(int dim, const double *u, const double *du, double gam)
{
    double rho, v[3], p;
    or_prim(dim, u, gam, &rho, v, &p);
    double drho = du[0];
    double rho1 = rho + drho;
    double mdm = 0.0, dm2 = 0.0, m2 = 0.0;
    for (int d = 0; d < dim; ++d) {
        mdm += u[1 + d] * du[1 + d];
        dm2 += du[1 + d] * du[1 + d];
        m2 += u[1 + d] * u[1 + d];
    }
    double dp = (gam - 1.0) * (du[dim + 1] - (mdm + 0.5 * dm2) / rho1 + drho * m2 / (2.0 * rho * rho1));
    double p1 = p + dp;
    return -drho * (log(p1) - gam * log(rho1)) - rho * (log1p(dp / p) - gam * log1p(drho / rho));
}

/* ------------------------------------------------------------------------ */
/* Ideal GLM-MHD (the second system of Sec. 4.1.1 and 4.3.3)                 */
/* ------------------------------------------------------------------------ */
/* u = (rho, rho v_1..3, E, B_1..3, psi), V = 9, in one or two space
 * dimensions (all three vector components kept: the "1.5D" form).
 *   p = (gamma-1) (E - rho |v|^2/2 - |B|^2/2 - psi^2/2)
 * Physical flux in direction n (GLM extension with cleaning speed c_h):
 *   f_rho = rho v_n
 *   f_m   = rho v v_n + (p + |B|^2/2) e_n - B B_n
 *   f_E   = v_n (rho |v|^2/2 + gamma p/(gamma-1) + |B|^2) - B_n (v.B) + c_h psi B_n
 *           (the psi^2/2 part of E is carried by the non-conservative term)
 *   f_B   = v_n B - B_n v + c_h psi e_n
 *   f_psi = c_h B_n
 * Non-conservative part (Powell term with the GLM transport of psi): the
 * system is u_t + sum_n [ d_n f_n + Phi(u) d_n B_n + Phi_n(u) d_n psi ] = 0 with
 *   Phi   = (0, B, v.B, v, 0)            (the Powell source, times div B)
 *   Phi_n = (0, 0, 0, 0, v_n psi, 0, 0, 0, v_n).                              */
static int or_mhd_prim(const double *u, double gam, double *rho, double *v, double *p, double *B, double *psi)
{
    for (int k = 0; k < 9; ++k)
        if (!isfinite(u[k])) return OR_ENONFINITE;
    *rho = u[0];
    if (!(*rho > 0.0)) return OR_ENONPHYS;
    double kin = 0.0, mag = 0.0;
    for (int d = 0; d < 3; ++d) {
        v[d] = u[1 + d] / u[0];
        kin += 0.5 * u[1 + d] * v[d];
        B[d] = u[5 + d];
        mag += 0.5 * B[d] * B[d];
    }
    *psi = u[8];
    *p = (gam - 1.0) * (u[4] - kin - mag - 0.5 * u[8] * u[8]);
    if (!(*p > 0.0)) return OR_ENONPHYS;
    return OR_OK;
}

void or_mhd_flux_phys(int dir, const double *u, double gam, double c_h, double *f)
{
    double rho, v[3], p, B[3], psi;
    or_mhd_prim(u, gam, &rho, v, &p, B, &psi);
    double vn = v[dir], Bn = B[dir], vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
    double ptot = p + 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    f[0] = rho * vn;
    for (int d = 0; d < 3; ++d) f[1 + d] = u[1 + d] * vn - B[d] * Bn + (d == dir ? ptot : 0.0);
    f[4] = vn * (u[4] - 0.5 * psi * psi + ptot) - Bn * vB + c_h * psi * Bn;
    for (int d = 0; d < 3; ++d) f[5 + d] = vn * B[d] - v[d] * Bn + (d == dir ? c_h * psi : 0.0);
    f[8] = c_h * Bn;
}

/* Entropy-conservative two-point flux for ideal GLM-MHD with the Powell term
 * (the Derigs et al. form of the Chandrashekar-type flux; the paper cites an
 * EC MHD flux without printing it).  With beta = rho / (2p), arithmetic means
 * {.}, logarithmic means {.}_log and p~ = {rho} / (2 {beta}):
 *   f_rho = {rho}_log {v_n}
 *   f_m   = f_rho {v} - (B_n,L B_R + B_n,R B_L)/2 + (p~ + (B_L.B_R)/2) e_n
 *   f_B   = {v_n B - B_n v} + c_h {psi} e_n
 *   f_psi = c_h {B_n}
 *   f_E   = f_rho ( 1/(2 (gamma-1) {beta}_log) - {|v|^2}/2 ) + f_m.{v} + f_B.{B}
 *           + f_psi {psi} - {v_n |B|^2}/2 + {B_n} {v.B} - c_h {psi B_n}         */
void or_mhd_flux_ec(int dir, const double *uL, const double *uR, double gam, double c_h, double *f)
{
    double rl, rr, vl[3], vr[3], pl, pr, Bl[3], Br[3], sl, sr;
    or_mhd_prim(uL, gam, &rl, vl, &pl, Bl, &sl);
    or_mhd_prim(uR, gam, &rr, vr, &pr, Br, &sr);
    double bl = 0.5 * rl / pl, br = 0.5 * rr / pr;
    double rho_log = or_logmean(rl, rr), beta_log = or_logmean(bl, br);
    double ptil = 0.5 * (rl + rr) / (bl + br);  /* {rho} / (2 {beta}) */
    double va[3], Ba[3], BB = 0.0, v2a = 0.0, vBl = 0.0, vBr = 0.0, B2l = 0.0, B2r = 0.0;
    for (int d = 0; d < 3; ++d) {
        va[d] = 0.5 * (vl[d] + vr[d]);
        Ba[d] = 0.5 * (Bl[d] + Br[d]);
        BB += Bl[d] * Br[d];
        v2a += 0.5 * (vl[d] * vl[d] + vr[d] * vr[d]);
        vBl += vl[d] * Bl[d];
        vBr += vr[d] * Br[d];
        B2l += Bl[d] * Bl[d];
        B2r += Br[d] * Br[d];
    }
    double psa = 0.5 * (sl + sr);
    double f0 = rho_log * va[dir];
    f[0] = f0;
    for (int d = 0; d < 3; ++d)
        f[1 + d] = f0 * va[d] - 0.5 * (Bl[dir] * Br[d] + Br[dir] * Bl[d]) + (d == dir ? ptil + 0.5 * BB : 0.0);
    for (int d = 0; d < 3; ++d)
        f[5 + d] = 0.5 * (vl[dir] * Bl[d] - vl[d] * Bl[dir] + vr[dir] * Br[d] - vr[d] * Br[dir])
                   + (d == dir ? c_h * psa : 0.0);
    f[8] = c_h * Ba[dir];
    double fe = f0 * (0.5 / ((gam - 1.0) * beta_log) - 0.5 * v2a);
    for (int d = 0; d < 3; ++d) fe += f[1 + d] * va[d] + f[5 + d] * Ba[d];
    fe += f[8] * psa;
    fe += -0.25 * (vl[dir] * B2l + vr[dir] * B2r) + Ba[dir] * 0.5 * (vBl + vBr)
          - c_h * 0.5 * (sl * Bl[dir] + sr * Br[dir]);
    f[4] = fe;
}

/* Fast magnetosonic speed in direction n:
 *   c_f^2 = (a^2 + |B|^2/rho + sqrt((a^2 + |B|^2/rho)^2 - 4 a^2 B_n^2/rho)) / 2,
 * a^2 = gamma p / rho. */
double or_mhd_cfast(int dir, const double *u, double gam)
{
    double rho, v[3], p, B[3], psi;
    or_mhd_prim(u, gam, &rho, v, &p, B, &psi);
    double a2 = gam * p / rho, b2 = (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]) / rho;
    double bn2 = B[dir] * B[dir] / rho;
    return sqrt(0.5 * (a2 + b2 + sqrt((a2 + b2) * (a2 + b2) - 4.0 * a2 * bn2)));
}

/* Local Lax-Friedrichs flux (f_L + f_R)/2 - lambda (u_R - u_L)/2,
 * lambda = max(|v_n| + c_f) over both sides. */
void or_mhd_flux_llf(int dir, const double *uL, const double *uR, double gam, double c_h, double *f)
{
    double fl[9], fr[9];
    or_mhd_flux_phys(dir, uL, gam, c_h, fl);
    or_mhd_flux_phys(dir, uR, gam, c_h, fr);
    double lam = fmax(fabs(uL[1 + dir] / uL[0]) + or_mhd_cfast(dir, uL, gam),
                      fabs(uR[1 + dir] / uR[0]) + or_mhd_cfast(dir, uR, gam));
    for (int k = 0; k < 9; ++k) f[k] = 0.5 * (fl[k] + fr[k]) - 0.5 * lam * (uR[k] - uL[k]);
}

/* Central flux (f_L + f_R)/2. */
void or_mhd_flux_central(int dir, const double *uL, const double *uR, double gam, double c_h, double *f)
{
    double fl[9], fr[9];
    or_mhd_flux_phys(dir, uL, gam, c_h, fl);
    or_mhd_flux_phys(dir, uR, gam, c_h, fr);
    for (int k = 0; k < 9; ++k) f[k] = 0.5 * (fl[k] + fr[k]);
}

/* Phi(u) and Phi_n(u) of the non-conservative part (see above). */
void or_mhd_nonconservative(int dir, const double *u, double gam, double *phi, double *phin)
{
    double rho, v[3], p, B[3], psi;
    or_mhd_prim(u, gam, &rho, v, &p, B, &psi);
    for (int k = 0; k < 9; ++k) phi[k] = phin[k] = 0.0;
    for (int d = 0; d < 3; ++d) {
        phi[1 + d] = B[d];
        phi[5 + d] = v[d];
    }
    phi[4] = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
    phin[4] = v[dir] * psi;
    phin[8] = v[dir];
}

/* Entropy s = -rho log(p / rho^gamma) with the MHD pressure (the same
 * mathematical entropy as for the Euler equations, Sec. 4.1.1). */
double or_mhd_entropy(const double *u, double gam)
{
    double rho, v[3], p, B[3], psi;
    or_mhd_prim(u, gam, &rho, v, &p, B, &psi);
    return -rho * (log(p) - gam * log(rho));
}

/* w = ds/du:
 *   w_rho = gamma - log(p rho^-gamma) - (gamma-1) rho |v|^2 / (2p)
 *   w_m = (gamma-1) rho v / p,  w_E = -(gamma-1) rho / p,
 *   w_B = (gamma-1) rho B / p,  w_psi = (gamma-1) rho psi / p.               */
void or_mhd_entropy_vars(const double *u, double gam, double *w)
{
    double rho, v[3], p, B[3], psi;
    or_mhd_prim(u, gam, &rho, v, &p, B, &psi);
    double rp = rho / p, v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    w[0] = gam - (log(p) - gam * log(rho)) - 0.5 * (gam - 1.0) * rp * v2;
    for (int d = 0; d < 3; ++d) {
        w[1 + d] = (gam - 1.0) * rp * v[d];
        w[5 + d] = (gam - 1.0) * rp * B[d];
    }
    w[4] = -(gam - 1.0) * rp;
    w[8] = (gam - 1.0) * rp * psi;
}

/* s(u + du) - s(u) without cancellation, as or_entropy_diff with
 *   dp = (gamma-1) [ dE - (m.dm + |dm|^2/2) / rho' + drho |m|^2 / (2 rho rho')
 *                    - (B.dB + |dB|^2/2) - (psi dpsi + dpsi^2/2) ]. */
double or_mhd_entropy_diff(const double *u, const double *du, double gam)
{
    double rho, v[3], p, B[3], psi;
    or_mhd_prim(u, gam, &rho, v, &p, B, &psi);
    double drho = du[0], rho1 = rho + drho;
    double mdm = 0.0, dm2 = 0.0, m2 = 0.0, BdB = 0.0, dB2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        mdm += u[1 + d] * du[1 + d];
        dm2 += du[1 + d] * du[1 + d];
        m2 += u[1 + d] * u[1 + d];
        BdB += B[d] * du[5 + d];
        dB2 += du[5 + d] * du[5 + d];
    }
    double dp = (gam - 1.0) * (du[4] - (mdm + 0.5 * dm2) / rho1 + drho * m2 / (2.0 * rho * rho1)
                               - (BdB + 0.5 * dB2) - (psi * du[8] + 0.5 * du[8] * du[8]));
    double p1 = p + dp;
    return -drho * (log(p1) - gam * log(rho1)) - rho * (log1p(dp / p) - gam * log1p(drho / rho));
}

/* ------------------------------------------------------------------------ */
/* Physics dispatch                                                          */
/* ------------------------------------------------------------------------ */

static int or_nvar(const or_mesh *m) { return m->physics == 1 ? 9 : m->dim + 2; }

static int or_node_ok(const or_mesh *m, const double *u)
{
    double rho, v[3], p, B[3], psi;
    if (m->physics == 1) return or_mhd_prim(u, m->gam, &rho, v, &p, B, &psi);
    return or_prim(m->dim, u, m->gam, &rho, v, &p);
}

static double or_node_entropy(const or_mesh *m, const double *u)
{
    return m->physics == 1 ? or_mhd_entropy(u, m->gam) : or_entropy(m->dim, u, m->gam);
}

static void or_node_entropy_vars(const or_mesh *m, const double *u, double *w)
{
    if (m->physics == 1) or_mhd_entropy_vars(u, m->gam, w);
    else or_entropy_vars(m->dim, u, m->gam, w);
}

static double or_node_entropy_diff(const or_mesh *m, const double *u, const double *du)
{
    return m->physics == 1 ? or_mhd_entropy_diff(u, du, m->gam) : or_entropy_diff(m->dim, u, du, m->gam);
}

/* ------------------------------------------------------------------------ */
/* Mesh helpers                                                              */
/* ------------------------------------------------------------------------ */

static int or_npe(int dim) { return dim == 2 ? 16 : 64; }
static int or_nelem(const or_mesh *m) { return m->n[0] * m->n[1] * (m->dim == 3 ? m->n[2] : 1); }

static const double *or_faces(const or_mesh *m, int d)
{
    const double *f = m->faces;
    for (int k = 0; k < d; ++k) f += m->n[k] + 1;
    return f;
}

static void or_elem_ijk(const or_mesh *m, int e, int *ix)
{
    ix[0] = e % m->n[0];
    ix[1] = (e / m->n[0]) % m->n[1];
    ix[2] = (m->dim == 3) ? e / (m->n[0] * m->n[1]) : 0;
}

static int or_elem_index(const or_mesh *m, const int *ix)
{
    return ix[0] + m->n[0] * (ix[1] + m->n[1] * ix[2]);
}

static double or_width(const or_mesh *m, int e, int d)
{
    int ix[3];
    or_elem_ijk(m, e, ix);
    const double *f = or_faces(m, d);
    return f[ix[d] + 1] - f[ix[d]];
}

/* Jacobian of the reference-to-physical map of a Cartesian element. */
static double or_jac(const or_mesh *m, int e)
{
    double J = 1.0;
    for (int d = 0; d < m->dim; ++d) J *= 0.5 * or_width(m, e, d);
    return J;
}

static void or_node_ijk(int l, int *il)
{
    il[0] = l % 4;
    il[1] = (l / 4) % 4;
    il[2] = l / 16;
}

static int or_node_index(const int *il) { return il[0] + 4 * (il[1] + 4 * il[2]); }

static void or_get(const or_mesh *m, const double *U, int e, int l, double *u)
{
    int ne = or_nelem(m), npe = or_npe(m->dim), V = or_nvar(m);
    for (int v = 0; v < V; ++v) u[v] = U[((size_t)v * ne + e) * npe + l];
}

static void or_put(const or_mesh *m, double *U, int e, int l, const double *u)
{
    int ne = or_nelem(m), npe = or_npe(m->dim), V = or_nvar(m);
    for (int v = 0; v < V; ++v) U[((size_t)v * ne + e) * npe + l] = u[v];
}

/* Quadrature weight of node l (tensor product of the 1D LGL weights). */
static double or_qnode(int dim, int l)
{
    double xi[4], q[4], D[16], Ds[16];
    or_lgl(xi, q, D, Ds);
    int il[3];
    or_node_ijk(l, il);
    double w = q[il[0]] * q[il[1]];
    if (dim == 3) w *= q[il[2]];
    return w;
}

/* Validate every node state of U. */
int or_check_state(const or_mesh *m, const double *U)
{
    int ne = or_nelem(m), npe = or_npe(m->dim);
    for (int e = 0; e < ne; ++e)
        for (int l = 0; l < npe; ++l) {
            double u[OR_MAXV];
            or_get(m, U, e, l, u);
            int st = or_node_ok(m, u);
            if (st) return st;
        }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Viscous shock (Sec. 4.3.2): exact solution and boundary states            */
/* ------------------------------------------------------------------------ */

/* Becker's viscous shock of the Navier-Stokes-Fourier equations at Pr = 3/4 in
 * Margolin's explicit form (Ma = 2 / sqrt(3 - gamma)), rho_0 = 1, shock speed
 * v = 1, viscosity mu, moving with the shock (x_0 = x - v t):
 *   c_0 = v / Ma, p_0 = c_0^2 rho_0 / gamma,
 *   l = 2 gamma (4/3 mu) / ((gamma+1) rho_0 v),
 *   chi = 2 exp(x_0 / (2 l)), w = 1 + (1 - sqrt(1 + 2 chi^2)) / (2 chi^2),
 *   rho = rho_0 / w, u = v (1 - w), p = p_0 / w (1 + (gamma-1)/2 Ma^2 (1 - w^2)).
 * The length scale is the one for which this profile solves the equations with
 * the Stokes stress (longitudinal viscosity 4/3 mu) and Pr = 3/4: the momentum
 * balance across the profile is -(4/3) mu w' = (gamma+1)/(2 gamma) (w-1)(w-1/2)/w,
 * and w above satisfies w' = -(w-1)(w-1/2)/(l w). */
void or_viscous_shock_prim(double x, double t, double gam, double mu, double *rho, double *u, double *p)
{
    const double rho0 = 1.0, v = 1.0;
    double Ma = 2.0 / sqrt(3.0 - gam);
    double c0 = v / Ma, p0 = c0 * c0 * rho0 / gam;
    double l = 2.0 * gam * (4.0 / 3.0 * mu) / ((gam + 1.0) * rho0 * v);
    double chi = 2.0 * exp((x - v * t) / (2.0 * l));
    double w = 1.0 + (1.0 - sqrt(1.0 + 2.0 * chi * chi)) / (2.0 * chi * chi);
    *rho = rho0 / w;
    *u = v * (1.0 - w);
    *p = p0 / w * (1.0 + 0.5 * (gam - 1.0) * Ma * Ma * (1.0 - w * w));
}

/* Conserved 2D state of the viscous shock (v_y = 0) at (x, m->time). */
static void or_viscous_shock_state(const or_mesh *m, double x, double *u)
{
    double rho, vx, p;
    or_viscous_shock_prim(x, m->time, m->gam, m->mu, &rho, &vx, &p);
    u[0] = rho;
    u[1] = rho * vx;
    u[2] = 0.0;
    u[3] = p / (m->gam - 1.0) + 0.5 * rho * vx * vx;
}

/* 1 when the face of element coordinates ix in direction d (right or left)
 * is a domain boundary of the viscous-shock set-up. */
static int or_x_boundary(const or_mesh *m, const int *ix, int d, int right)
{
    if (m->bc_x != 1 || d != 0) return 0;
    return right ? (ix[0] == m->n[0] - 1) : (ix[0] == 0);
}

/* ------------------------------------------------------------------------ */
/* Semidiscretisation F(U) on a set of elements                             */
/* ------------------------------------------------------------------------ */

/* For every node of every element with active[e] != 0:
 *   dU/dt = - sum_d (2/h_d) [ sum_{m != i_d} Dsplit[i_d][m] f#_d(u, u_m)
 *                             + (1/q_{i_d}) (delta_{i_d,3} f*_d(u, u+)
 *                                            - delta_{i_d,0} f*_d(u-, u)) ]
 * where u_m runs along the line of direction d through the node, u+ / u- are
 * the traces of the periodic neighbour across the right / left face, f# is
 * the EC volume flux and f* the selected surface flux.  active == NULL means
 * all elements.  Inactive elements' K entries are left untouched. */
static int or_mhd_rhs(const or_mesh *m, const double *U, const unsigned char *active, double *K);
static int or_ns_add_viscous(const or_mesh *m, const double *U, const unsigned char *active, double *K);
static int or_rhs_euler(const or_mesh *m, const double *U, const unsigned char *active, double *K);

int or_rhs(const or_mesh *m, const double *U, const unsigned char *active, double *K)
{
    if (m->physics == 1) return or_mhd_rhs(m, U, active, K);
    int status = or_rhs_euler(m, U, active, K);
    if (status == OR_OK && m->viscous) status = or_ns_add_viscous(m, U, active, K);
    return status;
}

/* The Euler part (inviscid flux divergence). */
static int or_rhs_euler(const or_mesh *m, const double *U, const unsigned char *active, double *K)
{
    double xi[4], q[4], D[16], Ds[16];
    or_lgl(xi, q, D, Ds);
    int dim = m->dim, V = dim + 2, npe = or_npe(dim), ne = or_nelem(m);
    int st = or_check_state(m, U);
    if (st) return st;
    for (int e = 0; e < ne; ++e) {
        if (active && !active[e]) continue;
        int ix[3];
        or_elem_ijk(m, e, ix);
        for (int l = 0; l < npe; ++l) {
            int il[3];
            or_node_ijk(l, il);
            double u[5], du[5] = { 0, 0, 0, 0, 0 };
            or_get(m, U, e, l, u);
            for (int d = 0; d < dim; ++d) {
                double scale = 2.0 / or_width(m, e, d);
                double acc[5] = { 0, 0, 0, 0, 0 };
                for (int mm = 0; mm < 4; ++mm) {
                    int jl[3] = { il[0], il[1], il[2] };
                    jl[d] = mm;
                    double um[5], f[5];
                    or_get(m, U, e, or_node_index(jl), um);
                    if (m->volume_integral == 1) {
                        /* weak form: the integral of l_i' f is, by LGL quadrature,
                           sum_m q_m D[m][i] f(u_m); divided by q_i (the mass matrix)
                           and with the sign of K = -(...) */
                        or_flux_phys(dim, d, um, m->gam, f);
                        for (int v = 0; v < V; ++v) acc[v] -= q[mm] * D[mm * 4 + il[d]] / q[il[d]] * f[v];
                    } else if (mm != il[d]) {
                        /* flux differencing along the line (Dsplit has a zero diagonal) */
                        or_flux_ec(dim, d, u, um, m->gam, f);
                        for (int v = 0; v < V; ++v) acc[v] += Ds[il[d] * 4 + mm] * f[v];
                    }
                }
                /* surface: right face (i_d = 3) and left face (i_d = 0) */
                if (il[d] == 3 || il[d] == 0) {
                    int right = (il[d] == 3);
                    int jx[3] = { ix[0], ix[1], ix[2] };
                    jx[d] = right ? (ix[d] + 1) % m->n[d] : (ix[d] + m->n[d] - 1) % m->n[d];
                    int jl[3] = { il[0], il[1], il[2] };
                    jl[d] = right ? 0 : 3;
                    double un[5], f[5];
                    if (or_x_boundary(m, ix, d, right)) {
                        /* viscous shock: inflow of the exact state on the left, outflow on the right */
                        if (right) for (int v = 0; v < V; ++v) un[v] = u[v];
                        else or_viscous_shock_state(m, or_faces(m, 0)[0], un);
                    } else {
                        or_get(m, U, or_elem_index(m, jx), or_node_index(jl), un);
                    }
                    if (right) {
                        or_surface_flux(m, d, u, un, f);
                        for (int v = 0; v < V; ++v) acc[v] += f[v] / q[3];
                    } else {
                        or_surface_flux(m, d, un, u, f);
                        for (int v = 0; v < V; ++v) acc[v] -= f[v] / q[0];
                    }
                }
                for (int v = 0; v < V; ++v) du[v] += scale * acc[v];
            }
            double k[5];
            for (int v = 0; v < V; ++v) k[v] = -du[v];
            or_put(m, K, e, l, k);
        }
    }
    return OR_OK;
}

/* GLM-MHD right-hand side (2D meshes; the third vector components are carried
 * along).  Per node and direction d, with the volume term (EC flux
 * differencing, or the standard weak form, by volume_integral), the surface
 * flux f* (EC, LLF or central by surface_flux) and the non-conservative part in
 * strong form with the interface averages of B_d and psi (the Powell term's
 * standard DGSEM discretisation):
 *   dU/dt = - sum_d (2/h_d) [ sum_{m != i} Dsplit[i][m] f#(u, u_m)   (or the weak form)
 *             + (1/q_i) (delta_i3 f*(u, u+) - delta_i0 f*(u-, u))
 *             + Phi(u) ( sum_m D[i][m] B_d,m + (1/q_i) (delta_i3 ({B_d}+ - B_d) - delta_i0 ({B_d}- - B_d)) )
 *             + Phi_d(u) ( the same with psi ) ]                             */
static void or_mhd_surface_flux(const or_mesh *m, int dir, const double *uL, const double *uR, double *f)
{
    if (m->surface_flux == 2) or_mhd_flux_llf(dir, uL, uR, m->gam, m->c_h, f);
    else if (m->surface_flux == 5) or_mhd_flux_central(dir, uL, uR, m->gam, m->c_h, f);
    else or_mhd_flux_ec(dir, uL, uR, m->gam, m->c_h, f);
}

static int or_mhd_rhs(const or_mesh *m, const double *U, const unsigned char *active, double *K)
{
    double xi[4], q[4], D[16], Ds[16];
    or_lgl(xi, q, D, Ds);
    int dim = m->dim, npe = or_npe(dim), ne = or_nelem(m);
    int st = or_check_state(m, U);
    if (st) return st;
    for (int e = 0; e < ne; ++e) {
        if (active && !active[e]) continue;
        int ix[3];
        or_elem_ijk(m, e, ix);
        for (int l = 0; l < npe; ++l) {
            int il[3];
            or_node_ijk(l, il);
            double u[9], du[9] = { 0 };
            or_get(m, U, e, l, u);
            for (int d = 0; d < dim; ++d) {
                double scale = 2.0 / or_width(m, e, d);
                double acc[9] = { 0 }, dB = 0.0, dpsi = 0.0;
                int t = il[d];
                for (int mm = 0; mm < 4; ++mm) {
                    int jl[3] = { il[0], il[1], il[2] };
                    jl[d] = mm;
                    double um[9], f[9];
                    or_get(m, U, e, or_node_index(jl), um);
                    dB += D[t * 4 + mm] * um[5 + d];
                    dpsi += D[t * 4 + mm] * um[8];
                    if (m->volume_integral == 1) {
                        /* weak form, as for the Euler equations */
                        or_mhd_flux_phys(d, um, m->gam, m->c_h, f);
                        for (int v = 0; v < 9; ++v) acc[v] -= q[mm] * D[mm * 4 + t] / q[t] * f[v];
                    } else if (mm != t) {
                        or_mhd_flux_ec(d, u, um, m->gam, m->c_h, f);
                        for (int v = 0; v < 9; ++v) acc[v] += Ds[t * 4 + mm] * f[v];
                    }
                }
                if (t == 3 || t == 0) {
                    int right = (t == 3);
                    int jx[3] = { ix[0], ix[1], ix[2] };
                    jx[d] = right ? (ix[d] + 1) % m->n[d] : (ix[d] + m->n[d] - 1) % m->n[d];
                    int jl[3] = { il[0], il[1], il[2] };
                    jl[d] = right ? 0 : 3;
                    double un[9], f[9];
                    or_get(m, U, or_elem_index(m, jx), or_node_index(jl), un);
                    double Bavg = 0.5 * (u[5 + d] + un[5 + d]), savg = 0.5 * (u[8] + un[8]);
                    if (right) {
                        or_mhd_surface_flux(m, d, u, un, f);
                        for (int v = 0; v < 9; ++v) acc[v] += f[v] / q[3];
                        dB += (Bavg - u[5 + d]) / q[3];
                        dpsi += (savg - u[8]) / q[3];
                    } else {
                        or_mhd_surface_flux(m, d, un, u, f);
                        for (int v = 0; v < 9; ++v) acc[v] -= f[v] / q[0];
                        dB -= (Bavg - u[5 + d]) / q[0];
                        dpsi -= (savg - u[8]) / q[0];
                    }
                }
                double phi[9], phin[9];
                or_mhd_nonconservative(d, u, m->gam, phi, phin);
                for (int v = 0; v < 9; ++v) du[v] += scale * (acc[v] + phi[v] * dB + phin[v] * dpsi);
            }
            double k[9];
            for (int v = 0; v < 9; ++v) k[v] = -du[v];
            or_put(m, K, e, l, k);
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Navier-Stokes-Fourier terms (BR1), 2D                                     */
/* ------------------------------------------------------------------------ */
/* Viscous flux in direction d from the velocity and the gradients g[dir][q] of
 * the primitive variables q = (rho, v_x, v_y, T), T = p / rho (gas constant 1),
 * Stokes hypothesis, heat conductivity kappa = gamma mu / ((gamma-1) Pr):
 *   tau_xx = mu (4/3 dv_x/dx - 2/3 dv_y/dy), tau_yy = mu (4/3 dv_y/dy - 2/3 dv_x/dx),
 *   tau_xy = mu (dv_x/dy + dv_y/dx),
 *   f_v,x = (0, tau_xx, tau_xy, v_x tau_xx + v_y tau_xy + kappa dT/dx), likewise in y. */
void or_ns_viscous_flux(int d, double vx, double vy, const double *g, double mu, double kappa, double *f)
{
    const double *gx = g, *gy = g + 4;
    double div = gx[1] + gy[2];
    double txx = mu * (2.0 * gx[1] - 2.0 / 3.0 * div);
    double tyy = mu * (2.0 * gy[2] - 2.0 / 3.0 * div);
    double txy = mu * (gy[1] + gx[2]);
    f[0] = 0.0;
    if (d == 0) {
        f[1] = txx;
        f[2] = txy;
        f[3] = vx * txx + vy * txy + kappa * gx[3];
    } else {
        f[1] = txy;
        f[2] = tyy;
        f[3] = vx * txy + vy * tyy + kappa * gy[3];
    }
}

static void or_ns_prim4(const double *u, double gam, double *q)
{
    double rho, v[3], p;
    or_prim(2, u, gam, &rho, v, &p);
    q[0] = rho;
    q[1] = v[0];
    q[2] = v[1];
    q[3] = p / rho;
}

/* Wall values of q at a boundary face of the viscous shock: the exact velocity
 * and temperature (moving isothermal no-slip wall), the density of the trace. */
static void or_ns_wall(const or_mesh *m, int right, const double *qown, double *qw)
{
    double x = right ? or_faces(m, 0)[m->n[0]] : or_faces(m, 0)[0];
    double rho, vx, p;
    or_viscous_shock_prim(x, m->time, m->gam, m->mu, &rho, &vx, &p);
    qw[0] = qown[0];
    qw[1] = vx;
    qw[2] = 0.0;
    qw[3] = p / rho;
}

/* BR1: (1) gradients of q per node in strong form with the face mean of q as
 * interface value (the wall values at a domain boundary),
 *   g_d = (2/h_d) [ sum_m D[i][m] q_m + (1/q_i) (delta_i3 (q*_+ - q) - delta_i0 (q*_- - q)) ];
 * (2) the divergence of the viscous flux in the same form with the face mean of
 * the two sides' viscous fluxes (at a domain boundary: the flux of the wall
 * velocity with the trace's gradient), added to K (u_t = ... + div f_v). */
static int or_ns_add_viscous(const or_mesh *m, const double *U, const unsigned char *active, double *K)
{
    double xi[4], q[4], D[16], Ds[16];
    or_lgl(xi, q, D, Ds);
    int npe = or_npe(2), ne = or_nelem(m);
    double kappa = m->gam * m->mu / ((m->gam - 1.0) * m->prandtl);
    double *G = (double *)malloc(sizeof(double) * (size_t)ne * npe * 8);
    if (!G) return OR_ENOMEM;
    for (int e = 0; e < ne; ++e) {
        int ix[3];
        or_elem_ijk(m, e, ix);
        for (int l = 0; l < npe; ++l) {
            int il[3];
            or_node_ijk(l, il);
            double u[4], qo[4];
            or_get(m, U, e, l, u);
            or_ns_prim4(u, m->gam, qo);
            for (int d = 0; d < 2; ++d) {
                double acc[4] = { 0, 0, 0, 0 };
                int t = il[d];
                for (int mm = 0; mm < 4; ++mm) {
                    int jl[3] = { il[0], il[1], il[2] };
                    jl[d] = mm;
                    double um[4], qm[4];
                    or_get(m, U, e, or_node_index(jl), um);
                    or_ns_prim4(um, m->gam, qm);
                    for (int k = 0; k < 4; ++k) acc[k] += D[t * 4 + mm] * qm[k];
                }
                if (t == 0 || t == 3) {
                    int right = (t == 3);
                    double qs[4];
                    if (or_x_boundary(m, ix, d, right)) {
                        or_ns_wall(m, right, qo, qs);
                    } else {
                        int jx[3] = { ix[0], ix[1], ix[2] };
                        jx[d] = right ? (ix[d] + 1) % m->n[d] : (ix[d] + m->n[d] - 1) % m->n[d];
                        int jl[3] = { il[0], il[1], il[2] };
                        jl[d] = right ? 0 : 3;
                        double un[4], qn[4];
                        or_get(m, U, or_elem_index(m, jx), or_node_index(jl), un);
                        or_ns_prim4(un, m->gam, qn);
                        for (int k = 0; k < 4; ++k) qs[k] = 0.5 * (qo[k] + qn[k]);
                    }
                    for (int k = 0; k < 4; ++k) acc[k] += (right ? 1.0 : -1.0) * (qs[k] - qo[k]) / q[t];
                }
                double sc = 2.0 / or_width(m, e, d);
                for (int k = 0; k < 4; ++k) G[(((size_t)e * npe + l) * 2 + d) * 4 + k] = sc * acc[k];
            }
        }
    }
    for (int e = 0; e < ne; ++e) {
        if (active && !active[e]) continue;
        int ix[3];
        or_elem_ijk(m, e, ix);
        for (int l = 0; l < npe; ++l) {
            int il[3];
            or_node_ijk(l, il);
            double u[4], qo[4], k[4];
            or_get(m, U, e, l, u);
            or_ns_prim4(u, m->gam, qo);
            or_get(m, K, e, l, k);
            const double *go = G + ((size_t)e * npe + l) * 8;
            for (int d = 0; d < 2; ++d) {
                double acc[4] = { 0, 0, 0, 0 }, fo[4];
                int t = il[d];
                or_ns_viscous_flux(d, qo[1], qo[2], go, m->mu, kappa, fo);
                for (int mm = 0; mm < 4; ++mm) {
                    int jl[3] = { il[0], il[1], il[2] };
                    jl[d] = mm;
                    int lm = or_node_index(jl);
                    double um[4], qm[4], fm[4];
                    or_get(m, U, e, lm, um);
                    or_ns_prim4(um, m->gam, qm);
                    or_ns_viscous_flux(d, qm[1], qm[2], G + ((size_t)e * npe + lm) * 8, m->mu, kappa, fm);
                    for (int c = 0; c < 4; ++c) acc[c] += D[t * 4 + mm] * fm[c];
                }
                if (t == 0 || t == 3) {
                    int right = (t == 3);
                    double fs[4];
                    if (or_x_boundary(m, ix, d, right)) {
                        double qw[4];
                        or_ns_wall(m, right, qo, qw);
                        or_ns_viscous_flux(d, qw[1], qw[2], go, m->mu, kappa, fs);
                    } else {
                        int jx[3] = { ix[0], ix[1], ix[2] };
                        jx[d] = right ? (ix[d] + 1) % m->n[d] : (ix[d] + m->n[d] - 1) % m->n[d];
                        int jl[3] = { il[0], il[1], il[2] };
                        jl[d] = right ? 0 : 3;
                        int en = or_elem_index(m, jx), ln = or_node_index(jl);
                        double un[4], qn[4], fn[4];
                        or_get(m, U, en, ln, un);
                        or_ns_prim4(un, m->gam, qn);
                        or_ns_viscous_flux(d, qn[1], qn[2], G + ((size_t)en * npe + ln) * 8, m->mu, kappa, fn);
                        for (int c = 0; c < 4; ++c) fs[c] = 0.5 * (fo[c] + fn[c]);
                    }
                    for (int c = 0; c < 4; ++c) acc[c] += (right ? 1.0 : -1.0) * (fs[c] - fo[c]) / q[t];
                }
                double sc = 2.0 / or_width(m, e, d);
                for (int c = 0; c < 4; ++c) k[c] += sc * acc[c];
            }
            or_put(m, K, e, l, k);
        }
    }
    free(G);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Integrals                                                                 */
/* ------------------------------------------------------------------------ */

/* Discrete total entropy H(U) = sum_e J_e sum_l q_l s(u_l). */
double or_total_entropy(const or_mesh *m, const double *U)
{
    int npe = or_npe(m->dim), ne = or_nelem(m);
    double H = 0.0;
    for (int e = 0; e < ne; ++e) {
        double J = or_jac(m, e), He = 0.0;
        for (int l = 0; l < npe; ++l) {
            double u[OR_MAXV];
            or_get(m, U, e, l, u);
            He += or_qnode(m->dim, l) * or_node_entropy(m, u);
        }
        H += J * He;
    }
    return H;
}

/* Discrete integrals of the conserved variables, out[v] = sum_e J_e sum_l q_l u_v. */
void or_total_conserved(const or_mesh *m, const double *U, double *out)
{
    int npe = or_npe(m->dim), ne = or_nelem(m), V = or_nvar(m);
    for (int v = 0; v < V; ++v) out[v] = 0.0;
    for (int e = 0; e < ne; ++e) {
        double J = or_jac(m, e);
        for (int v = 0; v < V; ++v) {
            double s = 0.0;
            for (int l = 0; l < npe; ++l) s += or_qnode(m->dim, l) * U[((size_t)v * ne + e) * npe + l];
            out[v] += J * s;
        }
    }
}

/* Entropy production <W(U), K> = sum_e J_e sum_l q_l w(u_l) . k_l
 * (EntropyChange_EntropyVariables_ReArranged without the dt b_i factor). */
double or_entropy_production(const or_mesh *m, const double *U, const double *K)
{
    int npe = or_npe(m->dim), ne = or_nelem(m), V = or_nvar(m);
    double s = 0.0;
    for (int e = 0; e < ne; ++e) {
        double J = or_jac(m, e), se = 0.0;
        for (int l = 0; l < npe; ++l) {
            double u[OR_MAXV], k[OR_MAXV], w[OR_MAXV];
            or_get(m, U, e, l, u);
            or_get(m, K, e, l, k);
            or_node_entropy_vars(m, u, w);
            double dot = 0.0;
            for (int v = 0; v < V; ++v) dot += w[v] * k[v];
            se += or_qnode(m->dim, l) * dot;
        }
        s += J * se;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Relaxation (Sec. 3.1)                                                     */
/* ------------------------------------------------------------------------ */

/* r(gamma) = H(U_n + gamma dt d) - H(U_n) - gamma dH + offset, evaluated as the
 * quadrature of the stable per-node entropy difference, and
 * r'(gamma) = <W(U_n + gamma dt d), dt d> - dH. */
void or_relax_eval(const or_mesh *m, const double *Un, const double *d, double dt, double gamma,
                   double dH, double offset, double *r, double *rp)
{
    int npe = or_npe(m->dim), ne = or_nelem(m), V = or_nvar(m);
    double sr = 0.0, srp = 0.0;
    for (int e = 0; e < ne; ++e) {
        double J = or_jac(m, e), er = 0.0, erp = 0.0;
        for (int l = 0; l < npe; ++l) {
            double u[OR_MAXV], dd[OR_MAXV], du[OR_MAXV], u1[OR_MAXV], w[OR_MAXV];
            or_get(m, Un, e, l, u);
            or_get(m, d, e, l, dd);
            for (int v = 0; v < V; ++v) {
                du[v] = gamma * dt * dd[v];
                u1[v] = u[v] + du[v];
            }
            or_node_entropy_vars(m, u1, w);
            double dot = 0.0;
            for (int v = 0; v < V; ++v) dot += w[v] * dt * dd[v];
            double ql = or_qnode(m->dim, l);
            er += ql * or_node_entropy_diff(m, u, du);
            erp += ql * dot;
        }
        sr += J * er;
        srp += J * erp;
    }
    *r = sr - gamma * dH + offset;
    *rp = srp - dH;
}

/* True when the candidate state U_n + gamma dt d is admissible at every node. */
static int or_candidate_ok(const or_mesh *m, const double *Un, const double *d, double dt, double gamma)
{
    int npe = or_npe(m->dim), ne = or_nelem(m), V = or_nvar(m);
    for (int e = 0; e < ne; ++e)
        for (int l = 0; l < npe; ++l) {
            double u[OR_MAXV], dd[OR_MAXV];
            or_get(m, Un, e, l, u);
            or_get(m, d, e, l, dd);
            for (int k = 0; k < V; ++k) u[k] += gamma * dt * dd[k];
            if (or_node_ok(m, u)) return 0;
        }
    return 1;
}

/* Solve r(gamma) = 0: Newton with unit step from opt->gamma0; accept the first
 * iterate with |r| <= tol_r.  If Newton fails, bisection on [bis_lo, bis_hi]
 * (the bracket is widened once to [bis_lo/2, 2 bis_hi] when r does not change
 * sign; gamma = 0, the trivial root, is never bracketed).  If that fails too,
 * gamma = 1 and the fallback flag (the paper's non-relaxed step). */
void or_relax_solve(const or_mesh *m, const double *Un, const double *d, double dt, double dH,
                    double offset, const or_relax *opt, or_info *info)
{
    double g = opt->gamma0, r = 0.0, rp = 0.0;
    int passes = 0, iters = 0;
    info->flags = 0;
    /* trivial direction: any gamma is a root */
    int npe = or_npe(m->dim), ne = or_nelem(m), V = or_nvar(m), nonzero = 0;
    for (size_t k = 0; k < (size_t)V * ne * npe; ++k)
        if (d[k] != 0.0) { nonzero = 1; break; }
    if (!nonzero) {
        info->gamma = 1.0;
        info->r = offset;
        info->passes = 0;
        info->newton_iters = 0;
        info->flags = OR_FLAG_TRIVIAL;
        return;
    }
    for (int k = 0; k < opt->max_newton; ++k) {
        if (!(g > 0.0) || !or_candidate_ok(m, Un, d, dt, g)) break;
        or_relax_eval(m, Un, d, dt, g, dH, offset, &r, &rp);
        ++passes;
        if (fabs(r) <= opt->tol_r) {
            info->gamma = g;
            info->r = r;
            info->passes = passes;
            info->newton_iters = iters;
            return;
        }
        if (!(rp != 0.0) || !isfinite(r) || !isfinite(rp)) break;
        double step = r / rp;
        g -= step;
        ++iters;
        if (fabs(step) < opt->tol_step) {
            /* no further progress possible at this precision */
            if (!(g > 0.0) || !or_candidate_ok(m, Un, d, dt, g)) break;
            or_relax_eval(m, Un, d, dt, g, dH, offset, &r, &rp);
            ++passes;
            if (fabs(r) <= opt->tol_r) {
                info->gamma = g;
                info->r = r;
                info->passes = passes;
                info->newton_iters = iters;
                return;
            }
            break;
        }
    }
    info->newton_iters = iters;
    /* bisection */
    info->flags |= OR_FLAG_BISECT;
    double lo = opt->bis_lo, hi = opt->bis_hi, rlo, rhi, dummy;
    for (int widen = 0; widen < 2; ++widen) {
        int ok_lo = or_candidate_ok(m, Un, d, dt, lo), ok_hi = or_candidate_ok(m, Un, d, dt, hi);
        if (ok_lo && ok_hi) {
            or_relax_eval(m, Un, d, dt, lo, dH, offset, &rlo, &dummy);
            or_relax_eval(m, Un, d, dt, hi, dH, offset, &rhi, &dummy);
            passes += 2;
            if (rlo < 0.0 && rhi > 0.0) {
                for (int k = 0; k < opt->max_bisect; ++k) {
                    double mid = 0.5 * (lo + hi), rm;
                    or_relax_eval(m, Un, d, dt, mid, dH, offset, &rm, &dummy);
                    ++passes;
                    if (fabs(rm) <= opt->tol_r) {
                        info->gamma = mid;
                        info->r = rm;
                        info->passes = passes;
                        return;
                    }
                    if (rm < 0.0) lo = mid;
                    else hi = mid;
                }
                break;
            }
        }
        lo = 0.5 * opt->bis_lo;
        hi = 2.0 * opt->bis_hi;
    }
    /* non-relaxed step */
    info->flags |= OR_FLAG_FALLBACK;
    info->gamma = 1.0;
    or_relax_eval(m, Un, d, dt, 1.0, dH, offset, &r, &rp);
    info->r = r;
    info->passes = passes;
}

/* ------------------------------------------------------------------------ */
/* Tableau                                                                   */
/* ------------------------------------------------------------------------ */

/* Dense Butcher matrix of level r: row i has c_i - a_{i,i-1} in column 1 and
 * a_{i,i-1} in column i-1 (for i = 2 both land in column 1 and sum to c_2). */
void or_dense_A(const or_tableau *t, int r, double *A)
{
    int S = t->S;
    memset(A, 0, sizeof(double) * S * S);
    for (int i = 1; i < S; ++i) {
        double a = t->a_sub[r * S + i];
        A[i * S + 0] += t->c[i] - a;
        A[i * S + (i - 1)] += a;
    }
}

/* Stage i (zero-based) is evaluated by level r iff i == 0 or i >= S - E_r + 1:
 * a level with E evaluations computes K_1 and K_{S-E+2}, ..., K_S. */
int or_stage_active(const or_tableau *t, int r, int i)
{
    return i == 0 || i >= t->S - t->E[r] + 1;
}

static int or_validate(const or_mesh *m, const or_tableau *t, const int *level)
{
    if (!(m->dim == 2 || m->dim == 3)) return OR_EINVAL;
    if (m->physics == 1 && m->dim != 2) return OR_EINVAL;
    if (m->viscous && (m->dim != 2 || m->physics != 0 || !(m->prandtl > 0.0) || !(m->mu >= 0.0))) return OR_EINVAL;
    if (t->S < 2 || t->S > OR_MAXS || t->R < 1 || t->R > OR_MAXR) return OR_EINVAL;
    for (int r = 0; r < t->R; ++r) {
        if (t->E[r] < 2 || t->E[r] > t->S) return OR_EINVAL;
        /* archetype structure: no sub-diagonal coupling into a stage the level
         * does not evaluate, nor into its first evaluated stage after K_1 */
        for (int i = 1; i <= t->S - t->E[r] + 1 && i < t->S; ++i)
            if (t->a_sub[r * t->S + i] != 0.0) return OR_EINVAL;
    }
    int ne = or_nelem(m);
    for (int e = 0; e < ne; ++e)
        if (level[e] < 0 || level[e] >= t->R) return OR_EINVAL;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* One step                                                                  */
/* ------------------------------------------------------------------------ */

static int or_finish_step(const or_mesh *m, const or_tableau *t, const or_relax *opt, double *U,
                          const double *d, double dt, double dH, or_info *info)
{
    size_t M = (size_t)or_nvar(m) * or_nelem(m) * or_npe(m->dim);
    info->dH = dH;
    info->H_old = or_total_entropy(m, U);
    if (opt->relax) {
        double offset = (opt->anchor == 1) ? (info->H_old - opt->H0) : 0.0;
        or_relax_solve(m, U, d, dt, dH, offset, opt, info);
    } else {
        info->gamma = 1.0;
        info->r = 0.0;
        info->passes = 0;
        info->newton_iters = 0;
        info->flags = 0;
    }
    for (size_t k = 0; k < M; ++k) U[k] = U[k] + info->gamma * dt * d[k];
    info->H_new = or_total_entropy(m, U);
    (void)t;
    return OR_OK;
}

/* Literal partitioned RK step (PartitionedRKSystem): every stage is evaluated
 * on every element, U_{n,i} = U_n + dt sum_j a^{(r)}_{ij} K_j with the dense
 * A^{(r)} of the element's level; d = sum_i b_i K_i; relaxation; update.
 * U is overwritten with U_{n+1} (relaxed solution at t_n + gamma dt). */
int or_step_dense(const or_mesh *m, const or_tableau *t, const int *level, const or_relax *opt,
                  double *U, double dt, or_info *info)
{
    int st = or_validate(m, t, level);
    if (st) return st;
    st = or_check_state(m, U);
    if (st) return st;
    int S = t->S, ne = or_nelem(m), npe = or_npe(m->dim), V = or_nvar(m);
    size_t M = (size_t)V * ne * npe;
    double *Kall = (double *)calloc(M * S, sizeof(double));
    double *Ui = (double *)malloc(M * sizeof(double));
    double *d = (double *)calloc(M, sizeof(double));
    double *A = (double *)malloc(sizeof(double) * S * S * t->R);
    if (!Kall || !Ui || !d || !A) {
        free(Kall); free(Ui); free(d); free(A);
        return OR_ENOMEM;
    }
    for (int r = 0; r < t->R; ++r) or_dense_A(t, r, A + (size_t)r * S * S);
    memset(info->e, 0, sizeof(info->e));
    for (int i = 0; i < S; ++i) {
        for (int v = 0; v < V; ++v)
            for (int e = 0; e < ne; ++e) {
                const double *Ar = A + (size_t)level[e] * S * S;
                for (int l = 0; l < npe; ++l) {
                    size_t idx = ((size_t)v * ne + e) * npe + l;
                    double s = 0.0;
                    for (int j = 0; j < i; ++j) s += Ar[i * S + j] * Kall[(size_t)j * M + idx];
                    Ui[idx] = U[idx] + dt * s;
                }
            }
        or_mesh ms = *m;
        ms.time = opt->t0 + t->c[i] * dt;  /* boundary values at the stage time */
        st = or_rhs(&ms, Ui, NULL, Kall + (size_t)i * M);
        if (st) break;
        if (t->b[i] != 0.0) info->e[i] = or_entropy_production(m, Ui, Kall + (size_t)i * M);
    }
    if (!st) {
        double dH = 0.0;
        for (int i = 0; i < S; ++i)
            if (t->b[i] != 0.0) {
                for (size_t k = 0; k < M; ++k) d[k] += t->b[i] * Kall[(size_t)i * M + k];
                dH += t->b[i] * info->e[i];
            }
        st = or_finish_step(m, t, opt, U, d, dt, dt * dH, info);
    }
    free(Kall); free(Ui); free(d); free(A);
    return st;
}

/* The same step in the form the paper's schemes are built for: only the
 * stages a level evaluates are computed on its elements (K_1 everywhere,
 * K_{S-E+2..S} on a level with E evaluations), and U_{n,i} is formed from
 * U_n, K_1 and K_{i-1} only; inactive levels take the cheap update
 * U_n + dt c_i K_1.  Two stage registers plus K_1 and K_{S-1} are kept. */
int or_step(const or_mesh *m, const or_tableau *t, const int *level, const or_relax *opt,
            double *U, double dt, or_info *info)
{
    int st = or_validate(m, t, level);
    if (st) return st;
    /* this form keeps K_1, K_{S-1} and K_S for d: other nonzero weights need the
       dense form (or_step_dense) */
    for (int i = 1; i < t->S - 2; ++i)
        if (t->b[i] != 0.0) return OR_EINVAL;
    st = or_check_state(m, U);
    if (st) return st;
    int S = t->S, ne = or_nelem(m), npe = or_npe(m->dim), V = or_nvar(m);
    size_t M = (size_t)V * ne * npe;
    double *K1 = (double *)calloc(M, sizeof(double));
    double *Kp = (double *)calloc(M, sizeof(double));
    double *Kc = (double *)calloc(M, sizeof(double));
    double *Ksm1 = (double *)calloc(M, sizeof(double));
    double *Ui = (double *)malloc(M * sizeof(double));
    double *d = (double *)calloc(M, sizeof(double));
    unsigned char *act = (unsigned char *)malloc(ne);
    if (!K1 || !Kp || !Kc || !Ksm1 || !Ui || !d || !act) {
        free(K1); free(Kp); free(Kc); free(Ksm1); free(Ui); free(d); free(act);
        return OR_ENOMEM;
    }
    memset(info->e, 0, sizeof(info->e));
    for (int i = 0; i < S && !st; ++i) {
        double *Kout = (i == 0) ? K1 : Kc;
        for (int e = 0; e < ne; ++e) {
            int r = level[e];
            double a = (i >= 1) ? t->a_sub[r * S + i] : 0.0;
            double a1 = (i >= 1) ? t->c[i] - a : 0.0;
            if (i == 1) { a1 = t->c[1]; a = 0.0; }
            act[e] = (unsigned char)or_stage_active(t, r, i);
            for (int v = 0; v < V; ++v)
                for (int l = 0; l < npe; ++l) {
                    size_t idx = ((size_t)v * ne + e) * npe + l;
                    double s = a1 * K1[idx];
                    if (a != 0.0) s += a * Kp[idx];
                    Ui[idx] = U[idx] + dt * s;
                }
        }
        or_mesh ms = *m;
        ms.time = opt->t0 + t->c[i] * dt;  /* boundary values at the stage time */
        st = or_rhs(&ms, Ui, act, Kout);
        if (st) break;
        if (t->b[i] != 0.0) info->e[i] = or_entropy_production(m, Ui, Kout);
        if (i == S - 2) memcpy(Ksm1, Kout, M * sizeof(double));
        if (i >= 1) {
            double *tmp = Kp;
            Kp = Kc;
            Kc = tmp;
        }
    }
    if (!st) {
        /* after the loop Kp holds K_S (S >= 2) */
        const double *KS = Kp;
        double dH = 0.0;
        for (size_t k = 0; k < M; ++k) {
            double s = t->b[S - 1] * KS[k];
            if (S >= 3 && t->b[S - 2] != 0.0) s += t->b[S - 2] * Ksm1[k];
            if (t->b[0] != 0.0) s += t->b[0] * K1[k];
            d[k] = s;
        }
        for (int i = 0; i < S; ++i)
            if (t->b[i] != 0.0) dH += t->b[i] * info->e[i];
        /* b may only be nonzero in positions 1, S-1, S for these archetypes */
        for (int i = 1; i < S - 2; ++i)
            if (t->b[i] != 0.0) st = OR_EINVAL;
        if (!st) st = or_finish_step(m, t, opt, U, d, dt, dt * dH, info);
    }
    free(K1); free(Kp); free(Kc); free(Ksm1); free(Ui); free(d); free(act);
    return st;
}
