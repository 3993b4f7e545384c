/*
 * perrk.h -- C ABI of libperrk: one Paired Explicit Relaxation Runge-Kutta
 * (P-ERRK) step of a degree-3 DGSEM discretisation of the compressible Euler
 * equations on periodic Cartesian meshes, on one AMD Instinct MI355X (gfx950).
 *
 * The method (arXiv 2507.04991):
 *   - Sec. 2.2: partitioned RK in Butcher form; each element belongs to one
 *     level r with E^(r) stage evaluations; the archetype tableaux of
 *     Appendix A (second, third, fourth order) with shared c and b and
 *     per-level sub-diagonal a^(r)_{i,i-1}; a level evaluates K_1 and
 *     K_{S-E+2}..K_S, inactive levels take the cheap update U_n + dt c_i K_1.
 *   - Sec. 2.4 and 3: relaxed update U_{n+1} = U_n + gamma dt d,
 *     d = sum_i b_i K_i, entropy change dH = dt sum_i b_i <W(U_{n,i}), K_i>
 *     accumulated stage by stage, gamma the root of
 *     r(gamma) = H(U_n + gamma dt d) - H(U_n) - gamma dH (Sec. 3.1), found by
 *     Newton with unit steps from the previous gamma; bisection, then the
 *     non-relaxed step gamma = 1, as fallbacks.
 *   - Sec. 2.1 / 4.1: DGSEM on Legendre-Gauss-Lobatto nodes with
 *     entropy-conservative flux differencing (Ranocha's EC/KEP two-point flux)
 *     in the volume; at faces the same flux or a dissipative one (Sec. 1 and
 *     the applications of Sec. 4-5): HLL with Davis wave speeds, local
 *     Lax-Friedrichs (Rusanov), HLLE (Einfeldt speeds), HLLC (Toro).
 *   - Sec. 2.3: entropy s(u) = -rho log(p / rho^gamma), H its quadrature.
 *
 * Data layout of every state array (caller's and library's): structure of
 * arrays [v][elem][node], node fastest; v = rho, rho v_1..rho v_dim, rho e
 * (V = dim + 2 fields; GLM-MHD: the nine fields listed at PERRK_SYSTEM_GLM_MHD);
 * node = i + 4 j (+ 16 k) with i along x; elements of a
 * case numbered ix + nx (iy + ny iz), cases concatenated.  Every pointer
 * named *_dev is device memory; everything else is host memory.
 *
 * Errors: every call returns a perrk_status.  Negative values are errors;
 * after an error perrk_last_error(ctx) describes it (when ctx exists).
 * Positive values are warnings (the call completed).  Calls never throw
 * across the boundary.  The library is thread-compatible, not thread-safe:
 * one context must not be used from two host threads at once.
 */
#ifndef PERRK_H
#define PERRK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct perrk_ctx perrk_ctx; /* opaque; owned by the library */

typedef enum {
    PERRK_OK = 0,
    PERRK_EINVAL = -1,      /* invalid argument or descriptor; no side effects */
    PERRK_ENOMEM = -2,      /* device or host allocation failed */
    PERRK_EHIP = -3,        /* a HIP runtime call failed (e.g. no GPU) */
    PERRK_ENONPHYS = -4,    /* rho <= 0 or p <= 0 in a state the step formed; u left unmodified */
    PERRK_ENONFINITE = -5,  /* NaN or Inf in a state the step formed; u left unmodified */
    PERRK_WARN_FALLBACK = 1 /* some case took the non-relaxed step gamma = 1 (see flags) */
} perrk_status;

/* Surface fluxes.  EC: Ranocha's entropy-conservative flux.  HLL: two waves,
 * speeds min/max(v_n -+ c) of both sides (Davis).  LLF: central flux minus
 * lambda (u_R - u_L) / 2, lambda = max(|v_n| + c) of both sides.  HLLE: HLL
 * with the Davis speeds widened by the Roe-averaged v_n -+ c (Einfeldt).
 * HLLC: three waves with the Davis outer speeds and Toro's contact speed and
 * star states.  All but EC dissipate entropy. */
enum { PERRK_FLUX_EC = 0, PERRK_FLUX_HLL = 1, PERRK_FLUX_LLF = 2, PERRK_FLUX_HLLE = 3, PERRK_FLUX_HLLC = 4,
       PERRK_FLUX_CENTRAL = 5 /* (f_L + f_R)/2: GLM-MHD only */ };
/* Volume term.  FLUX_DIFFERENCING: split form with Ranocha's EC two-point flux
 * (Sec. 4.1; entropy conservative with the EC surface flux).  WEAK: the
 * standard weak-form volume integral (the linear-invariant test of Sec. 4.2),
 * evaluated as the split form with the central two-point flux, which the SBP
 * property of the LGL derivative matrix makes identical to it. */
enum { PERRK_VOLUME_FLUX_DIFFERENCING = 0, PERRK_VOLUME_WEAK = 1 };
/* System of conservation laws.  EULER: compressible Euler, V = dim + 2 fields
 * (rho, rho v_1..rho v_dim, rho e).  GLM_MHD: ideal MHD with generalised
 * Lagrange multiplier divergence cleaning (the second system of Sec. 4.1.1 and
 * 4.3.3), 2D meshes only, V = 9 fields (rho, rho v_1..3, E, B_1..3, psi; all
 * three vector components are carried, so a mesh with no variation in y gives
 * the "1.5D" problems), PERRK_FP64 only.  Its system adds the Powell term
 * Phi(u) div B, Phi = (0, B, v.B, v, 0), and the GLM transport
 * v_d psi (0, 0, 0, 0, psi, 0, 0, 0, 1) d_d psi to the flux divergence; the
 * cleaning speed c_h is glm_ch.  Surface fluxes: EC, LLF (fast magnetosonic
 * speeds) or CENTRAL; volume term: EC flux differencing or WEAK.  The entropy
 * is the same s = -rho log(p rho^-gamma) with the MHD pressure
 * p = (gamma-1)(E - rho |v|^2/2 - |B|^2/2 - psi^2/2). */
enum { PERRK_SYSTEM_EULER = 0, PERRK_SYSTEM_GLM_MHD = 1 };
/* FP64: every operation in double precision.
 * MIXED: the stages with b_i = 0 compute volume and surface fluxes in single
 * precision with single-precision accumulation, form their stage states in
 * single precision and store K_i in single precision; the stages with
 * b_i != 0 (those entering d and the entropy change dH) run in double
 * precision; d, entropy sums and the gamma solve are double precision.
 * MIXED_ALL: every stage in single precision as above; d and the stage
 * entropy production are accumulated in double precision from the
 * single-precision K_i, and the gamma solve is double precision, so gamma is
 * the certified root of r for those K_i (entropy is then conserved to the
 * single-precision rounding of the K_i rather than to double rounding). */
enum { PERRK_FP64 = 0, PERRK_MIXED = 1, PERRK_MIXED_ALL = 2 };
/* STEP: r anchored to H(U_n) (first equality of the discrete entropy balance);
 * INITIAL: to H(U_0), the entropy of the first state stepped (its offset is
 * part of the relaxation state, see perrk_get_relaxation_state). */
enum { PERRK_ANCHOR_STEP = 0, PERRK_ANCHOR_INITIAL = 1 };
/* Initial guess of the Newton iteration: previous accepted gamma (1 at the
 * first step), the learned guess (perrk_set_guess_model), or the linear
 * extrapolation of the root history, 1 + 2 (gamma*_{n-1} - 1) - (gamma*_{n-2} - 1)
 * (see perrk_get_relaxation_state), once a case has taken two steps; an
 * extrapolation that is not finite, moves the previous root by 0.1 or more, or
 * is <= 0 is ignored (the previous accepted gamma is used).  Not in the paper:
 * Newton and bisection still decide the accepted gamma. */
enum { PERRK_GUESS_PREV = 0, PERRK_GUESS_MLP = 1, PERRK_GUESS_EXTRAP = 2 };
/* Per-case step flags (perrk_step_info.flags). */
enum {
    PERRK_FLAG_BISECT = 1,   /* Newton failed, bisection was used */
    PERRK_FLAG_FALLBACK = 2, /* no root found: gamma = 1 was taken */
    PERRK_FLAG_TRIVIAL = 4   /* d == 0 everywhere: gamma = 1 without a solve */
};

typedef struct {
    int32_t dim;               /* 2 or 3 */
    int32_t n_cases;           /* >= 1: independent meshes advanced together */
    const int32_t *n_elem_dir; /* [n_cases][3] elements per direction, >= 2 each (third = 1 in 2D);
                                  all cases together fewer than 2^29 nodes (elements x 4^dim),
                                  so that an FP64 field spans less than 4 GiB and the byte
                                  offset of a node in it fits in 32 bits: at most 2^25 - 1
                                  quadrilaterals or 2^23 - 1 hexahedra; larger meshes are
                                  rejected with PERRK_EINVAL */
    const double *face_coords; /* per case, per direction: n+1 increasing face positions, concatenated;
                                  the domain is periodic in every direction */
    double gas_gamma;          /* ratio of specific heats (> 1) */
    int32_t surface_flux;      /* PERRK_FLUX_EC .. PERRK_FLUX_HLLC */
    int32_t precision;         /* PERRK_FP64, PERRK_MIXED or PERRK_MIXED_ALL */
    int32_t volume_integral;   /* PERRK_VOLUME_FLUX_DIFFERENCING or PERRK_VOLUME_WEAK */
    int32_t system;            /* PERRK_SYSTEM_EULER or PERRK_SYSTEM_GLM_MHD */
    double glm_ch;             /* GLM-MHD divergence-cleaning speed (>= 0); ignored for Euler */
    int32_t viscous;           /* 1: add the Navier-Stokes-Fourier terms (Sec. 4.3.2): Stokes stress
                                  with viscosity mu, heat flux -kappa grad T, T = p / rho,
                                  kappa = gamma mu / ((gamma-1) prandtl), discretised by BR1
                                  (gradients of rho, v, T and the viscous flux with face means);
                                  Euler system, dim = 2 and PERRK_FP64 only */
    double mu, prandtl;        /* viscosity (>= 0) and Prandtl number (> 0) when viscous */
    int32_t bc_x;              /* 0: periodic; 1: the viscous-shock set-up of Sec. 4.3.2 (one case,
                                  viscous): at the left x end the exact shock state flows in, the
                                  right x end is a free outflow, and both are moving isothermal
                                  walls for the viscous terms (exact velocity and temperature of
                                  the shock with rho_0 = 1, speed 1, Ma = 2/sqrt(3-gamma), Pr 3/4,
                                  at the stage time t_n + c_i dt); y stays periodic */
} perrk_mesh_desc;

typedef struct {
    int32_t n_levels;          /* must equal the tableau's n_levels */
    const int32_t *elem_level; /* [total elements] level index 0..n_levels-1 (natural order) */
} perrk_partition_desc;

typedef struct {
    int32_t order;             /* 2, 3 or 4 */
    int32_t S;                 /* stages, 2..64 */
    int32_t n_levels;          /* 1..16 */
    const int32_t *E;          /* [n_levels] stage evaluations, 2..S */
    const double *c;           /* [S] abscissae shared by all levels */
    const double *b;           /* [S] weights shared by all levels, >= 0; at most 8 nonzero, and every
                                  level must evaluate each stage i > 1 with b_i != 0 (the archetypes
                                  have b_i != 0 only at i = 1, S-1, S; classic RK4 has four) */
    const double *a_sub;       /* [n_levels][S]: a^(r)_{i,i-1}; a^(r)_{i,1} = c_i - a^(r)_{i,i-1}.
                                  Must vanish for stages a level skips and for its first
                                  evaluated stage after K_1. */
} perrk_tableau_desc;

typedef struct {
    int32_t relax;             /* 0: plain P-ERK step (gamma = 1), 1: relaxation */
    int32_t max_newton;        /* Newton evaluations before bisection (>= 0) */
    double tol_r;              /* accept gamma only when |r(gamma)| <= tol_r */
    double tol_step;           /* a Newton step below this ends Newton after one more check */
    int32_t anchor;            /* PERRK_ANCHOR_STEP or PERRK_ANCHOR_INITIAL */
    int32_t max_bisect;        /* bisection steps before gamma = 1 (>= 0) */
    double bisect_lo, bisect_hi; /* bracket, 0 < lo < 1 < hi; widened once to [lo/2, 2 hi] */
    int32_t guess;             /* PERRK_GUESS_PREV, PERRK_GUESS_MLP or PERRK_GUESS_EXTRAP */
    int32_t fast_passes;       /* residual passes launched without host involvement (1..16);
                                  further passes run in one per-case completion kernel */
    int32_t use_graph;         /* 1: capture each step's launch sequence into a hipGraph */
    int32_t tune;              /* 1: at the first perrk_step, time every stage launch with 1, 2, 4 and 8
                                  wavefronts per workgroup on the caller's state and keep the fastest
                                  per stage (results do not depend on the choice); 0: 4 for all
                                  (1 for GLM-MHD, 2 for Navier-Stokes); -w (w = 1, 2, 4, 8): w for
                                  all (PERRK_EINVAL from perrk_init if that needs more LDS per
                                  workgroup than the device has) */
    int32_t tile;              /* element tiles the active lists keep together: 0 = chosen by the
                                  autotuner with tune = 1 (tile 1 otherwise); 1..PERRK_TILES fixed:
                                  2D tiles of 32 quadrilaterals (a full workgroup) 8x4, 4x8, 16x2,
                                  32x1; 3D cubes of 8^3, 4^3, 16^3 hexahedra, or whole rows.  Results
                                  do not depend on the tile. */
    int32_t phases;            /* Euler with the EC surface flux and flux differencing, and GLM-MHD:
                                  0 = chosen per stage with double-precision fluxes by the autotuner
                                  with tune = 1 (1 otherwise); 1 = a stage forms the pair fluxes of
                                  two directions per phase (Euler 2D: x and y, faces in a round of
                                  their own; 3D: z with the z faces, then x and y; GLM-MHD: x and y
                                  after the faces); 2 = one direction at a time (Euler: each with its
                                  faces, 2D: x, y; 3D: z, x, y; GLM-MHD: x, then y, after the faces),
                                  with half the pair-flux LDS per element.  Ignored by the other
                                  configurations.  Results do not depend on the choice. */
} perrk_options;
#define PERRK_TILES 4

typedef struct {
    double gamma;      /* accepted relaxation parameter; the solution is at t_n + gamma dt */
    double r;          /* relaxation residual at the accepted gamma */
    double dH;         /* dt sum_i b_i <W(U_{n,i}), K_i> */
    double H_delta;    /* H(U_{n+1}) - H(U_n) as integrated by the residual */
    double e[8];       /* <W(U_{n,i}), K_i> of the stages with b_i != 0, in stage order (at most 8) */
    double t;          /* accumulated relaxed time sum gamma dt since init */
    int32_t passes;    /* residual evaluations (full-mesh reductions) of the solve */
    int32_t flags;     /* PERRK_FLAG_* */
} perrk_step_info;

/* Default options: relax = 1, max_newton = 10, tol_r = 1e-12, tol_step = 1e-15,
 * anchor = STEP, max_bisect = 60, bracket [0.8, 1.2], guess = PREV,
 * fast_passes = 3, use_graph = 1, tune = 1, tile = 0, phases = 0. */
void perrk_default_options(perrk_options *opts);

/* Validates every descriptor on the host (no GPU call): tableau structure,
 * internal consistency sum_j a_ij = c_i (Sec. 2.2), shared b (conservation),
 * order conditions up to `order`, level and mesh ranges.  Returns PERRK_OK or
 * PERRK_EINVAL and writes a message into msg (may be NULL). */
int perrk_validate(const perrk_mesh_desc *mesh, const perrk_partition_desc *part,
                   const perrk_tableau_desc *tab, const perrk_options *opts, char *msg,
                   size_t msg_len);

/* Creates a context: validates (as perrk_validate), builds element tables and
 * the level-sorted active lists, allocates the stage registers and reduction
 * buffers on the current HIP device, and binds `stream` (hipStream_t; NULL =
 * default stream) for all later work.  Host descriptors may be freed after
 * return.  On error *out is NULL. */
int perrk_init(const perrk_mesh_desc *mesh, const perrk_partition_desc *part,
               const perrk_tableau_desc *tab, const perrk_options *opts, void *stream,
               perrk_ctx **out);

/* One P-ERRK step of every case, in place on u_dev (FP64, layout above,
 * caller-owned).  dt: [n_cases] host array of step sizes (> 0).  Work is
 * enqueued on the context's stream.  Every step reads u_dev afresh (in the
 * mixed modes its first stage also writes the library's single-precision copy
 * of U_n that the later single-precision stages read), so the caller may
 * change u_dev between steps.  info: [n_cases] host array or NULL; with
 * NULL the call does not synchronise; with info the call waits for the step
 * and fills it.  A step that forms a non-physical (rho <= 0 or p <= 0) or
 * non-finite stage state in any case is rejected: u_dev is left unmodified
 * and so is the state carried to the next step (t, gamma history, entropy
 * offset; see perrk_get_relaxation_state).  A step with info reports its own
 * rejection as PERRK_ENONPHYS or PERRK_ENONFINITE; the rejection of a step
 * called with info = NULL is reported, with the same codes, by the next step
 * called with info (whose own result is then valid and in info; the message
 * says which step failed).  Each step starts afresh: an earlier rejection
 * never makes a later step skip its update. */
int perrk_step(perrk_ctx *ctx, void *u_dev, const double *dt, perrk_step_info *info);

/* H[c] = discrete total entropy of case c of u_dev: sum over elements of
 * J_e sum_nodes q s(u) (Sec. 2.3).  Synchronises.  H: [n_cases] host.
 * Returns PERRK_ENONPHYS if a node has rho <= 0 or p <= 0, PERRK_ENONFINITE
 * if a node or a sum is not finite (H is still written); such an error
 * concerns this call only and never affects a later step. */
int perrk_entropy(perrk_ctx *ctx, const void *u_dev, double *H);

/* k_dev = F(u_dev) on every element: the semidiscretisation the stages
 * evaluate.  k_dev has the stage storage type: double (FP64) or float
 * (MIXED, MIXED_ALL: single-precision fluxes), same layout as u_dev.
 * Asynchronous on the context's stream.  A non-physical u_dev is not
 * reported (k_dev then holds whatever the fluxes give) and never affects a
 * later step. */
int perrk_rhs(perrk_ctx *ctx, const void *u_dev, void *k_dev);

/* Per-case state that one step hands to the next: the previous accepted gamma
 * (the Newton starting value), the accumulated entropy offset H(U_n) - H(U_0)
 * used by PERRK_ANCHOR_INITIAL, the relaxed time t, the last three roots
 * gamma* - 1 (most recent first: each step's accepted gamma moved by one more
 * Newton step -r/r' when Newton accepted it; the history of the learned guess)
 * and the number of accepted steps (the learned guess is used from the fourth
 * step on).
 * Read or restore (checkpoint / resume: a context restored from these values
 * continues bitwise as the one they were read from).  Host arrays, each may be
 * NULL (not read / not changed): gamma_prev, h_offset, t, n_steps [n_cases],
 * gamma_hist [n_cases][3].  Set: gamma_prev must be finite and > 0 and
 * n_steps >= 0, else PERRK_EINVAL with nothing changed.  Both synchronise. */
int perrk_get_relaxation_state(perrk_ctx *ctx, double *gamma_prev, double *h_offset, double *t,
                               double *gamma_hist, int32_t *n_steps);
int perrk_set_relaxation_state(perrk_ctx *ctx, const double *gamma_prev, const double *h_offset,
                               const double *t, const double *gamma_hist, const int32_t *n_steps);

/* Learned initial guess (guess = PERRK_GUESS_MLP): a multilayer perceptron
 * 8 -> 32 -> 32 -> 1 (tanh hidden layers), float32, predicting the increment
 * gamma*_n - gamma*_{n-1} of the root of each case (the root history of
 * perrk_get_relaxation_state).  weights: 1379 values, the 1377 network
 * parameters W1[32][8], b1[32], W2[32][32], b2[32], W3[1][32], b3[1] followed
 * by the output scale and shift.  Features per case, formed in double
 * precision: the last two increments of the root (gamma*_{n-1} - gamma*_{n-2},
 * gamma*_{n-2} - gamma*_{n-3}), gamma*_{n-1} - 1, dt, and the
 * entropy-production terms of this step's stages with b_i != 0 that come
 * before the last stage, divided by the sum of their magnitudes (padded with
 * zeros to four); each feature is normalised as (x - mean[k]) * scale[k].  The
 * first evaluation point is gamma*_{n-1} + shift + scale_out * network output;
 * a prediction that is not finite, has magnitude >= 0.1 or would make gamma
 * <= 0 is ignored (the previous accepted gamma is used).  The network is used once a case has taken three
 * steps.  Newton/bisection still decide the accepted gamma.  Host arrays;
 * copied. */
int perrk_set_guess_model(perrk_ctx *ctx, const float *weights, const float *mean,
                          const float *scale);

/* Training and inference of the same network on device arrays, asynchronous
 * on `stream` (hipStream_t, NULL = default); no allocation.
 * perrk_mlp_forward: y[n] = network(w, x[n][8]) (w: the 1377 parameters).
 * perrk_mlp_loss_grad: grad[1377] = d/dw of the mean squared error
 *   (1/n) sum (y_i - t_i)^2 and *loss_dev = that error (double, device; may be
 *   NULL); work_dev must hold perrk_mlp_workspace_bytes(n) bytes.  Sums are
 *   taken in a fixed order (bitwise reproducible).
 * perrk_mlp_adam: one Adam update of w[1377] with first/second moment arrays
 *   m, v (device, caller-initialised to 0) at step >= 1. */
size_t perrk_mlp_workspace_bytes(int64_t n);
int perrk_mlp_forward(const float *w_dev, const float *x_dev, int64_t n, float *y_dev, void *stream);
int perrk_mlp_loss_grad(const float *w_dev, const float *x_dev, const float *t_dev, int64_t n,
                        float *grad_dev, double *loss_dev, void *work_dev, size_t work_bytes,
                        void *stream);
/* perrk_mlp_loss_grad without a workspace, for callers that cannot allocate
 * device memory (code under stream capture, tight loops, harnesses that forbid
 * allocation): the same kernels and the same result, bit for bit, as
 * perrk_mlp_loss_grad, with the per-chunk partial sums in a static array of
 * the library (one per device, 11.3 MB, held until the process ends) instead
 * of work_dev.  Allocates nothing.  n must be in 1..PERRK_MLP_STATIC_MAX_N;
 * larger n returns PERRK_ENOMEM (use perrk_mlp_loss_grad), null pointers or
 * n <= 0 PERRK_EINVAL.  Every call on one device shares that array: calls that
 * overlap on one device (different streams, or threads) race and must be
 * ordered by the caller.  Asynchronous on `stream`. */
#define PERRK_MLP_STATIC_MAX_N 131072
int perrk_mlp_loss_grad_static(const float *w_dev, const float *x_dev, const float *t_dev, int64_t n,
                               float *grad_dev, double *loss_dev, void *stream);
int perrk_mlp_adam(float *w_dev, const float *grad_dev, float *m_dev, float *v_dev, int32_t step,
                   float lr, float beta1, float beta2, float eps, void *stream);

/* Kernel classes of the per-launch statistics. */
enum {
    PERRK_K_STAGE_FIRST = 0, /* stage 1: K_1 = F(U_n) on every element */
    PERRK_K_STAGE_MID = 1,   /* stages 2..S-1 on their active elements */
    PERRK_K_STAGE_LAST = 2,  /* stage S, writes the direction d */
    PERRK_K_RESIDUAL = 3,    /* relaxation residual passes (full mesh) */
    PERRK_K_SOLVER = 4,      /* per-case reductions and the Newton / bisection updates */
    PERRK_K_UPDATE = 5,      /* U_{n+1} = U_n + gamma dt d */
    PERRK_K_CLASSES = 6
};

/* Accumulated statistics of one kernel class: summed launch durations
 * (HIP events around each launch on the library's stream), summed algorithmic
 * bytes (compulsory HBM traffic of the launch: the arrays it must read and
 * write once; neighbour face reads are not counted) and launch count. */
typedef struct {
    double ms;
    double bytes;
    int64_t launches;
} perrk_kernel_stat;

/* on = 1: later steps are launched without the graph, each launch bracketed by
 * HIP events, and every step synchronises; on = 0 restores normal launches. */
int perrk_set_profiling(perrk_ctx *ctx, int on);

/* Copies the statistics of the PERRK_K_CLASSES classes into stats[] and, if
 * reset != 0, clears them. */
int perrk_get_kernel_stats(perrk_ctx *ctx, perrk_kernel_stat *stats, int reset);

/* Copies per-stage statistics (entry i = stage i + 1, n_stages = S entries)
 * collected while profiling into stats[] and, if reset != 0, clears them. */
int perrk_get_stage_stats(perrk_ctx *ctx, perrk_kernel_stat *stats, int n_stages, int reset);

/* Writes a short text describing the launch configuration in use (and, after
 * autotuning, the candidate timings). */
int perrk_get_tuning(perrk_ctx *ctx, char *buf, size_t len);

/* Last error message of ctx ("" if none). */
const char *perrk_last_error(const perrk_ctx *ctx);

/* Library version string. */
const char *perrk_version(void);

/* Frees every resource of ctx (waits for its stream first).  NULL is allowed. */
void perrk_destroy(perrk_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PERRK_H */
