// Internal declarations shared by the host side (perrk_host.cpp) and the
// kernels (perrk_kernels.hip) of libperrk.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "perrk.h"

#define PERRK_MAXR 16        // levels (a level index fits in 4 bits)
#define PERRK_NBR_MASK 0x0FFFFFFF
#define PERRK_NBR_SHIFT 28
#define PERRK_MAXS 64        // stages
#define PERRK_MAXB 8         // stages with b_i != 0 (entropy-production slots)
#define PERRK_RED_THREADS 1024  // block size of every per-case reduction (fixed: results depend on it)
#define PERRK_MLP_NW 1377

// Words of the device error array (bit 1: rho <= 0 or p <= 0, bit 2: non-finite).
enum {
    ERR_STEP = 0,     // errors of the step in flight; cleared as each step starts
    ERR_PENDING = 1,  // errors of steps not yet reported; cleared when a step with info reports them
    ERR_RHS = 2,      // written by perrk_rhs, never read
    ERR_ENTROPY = 3,  // errors of perrk_entropy; cleared as it starts
    ERR_WORDS = 4
};

// Node arrays are addressed by buffer instructions with one 32-bit byte range
// per field.  An FP64 field of n nodes spans 8 n bytes, so every case together
// must hold fewer than 2^29 nodes: at exactly 2^29 the range 2^32 no longer
// fits 32 bits.  The host rejects larger meshes (perrk_node_count_ok); the
// kernels build ranges with perrk_buffer_range, which saturates rather than
// wraps, so even a range computed past the limit never reads as zero.
#define PERRK_MAX_NODES (((int64_t)1 << 29) - 1)

__host__ __device__ constexpr bool perrk_node_count_ok(int64_t nodes)
{
    return nodes >= 0 && nodes <= PERRK_MAX_NODES;
}

__host__ __device__ constexpr uint32_t perrk_buffer_range(uint64_t elems, uint64_t elem_bytes)
{
    return elems * elem_bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)(elems * elem_bytes);
}

// Per-element geometry and bookkeeping (natural element order, all cases).
struct ElemInfo {
    int32_t nbr[6];     // periodic neighbours -x, +x, -y, +y, -z, +z: global element index in
                        // bits 0..27, the neighbour's level in bits 28..31 (same case)
    int32_t level;      // level index r
    int32_t case_id;    // owning case
    double metric[3];   // 2 / h_d
    double jac;         // prod_d h_d / 2
};

// Entry of a stage's active-element list: the element with its level, its case,
// and its neighbour words (as in ElemInfo::nbr), so that one load of 32 bytes
// gives a lane everything the addresses and coefficients of its own and its
// neighbours' nodes depend on.
struct __attribute__((aligned(32))) ActiveEntry {
    int32_t elem_level;  // element index | level << PERRK_NBR_SHIFT
    int32_t case_id;
    int32_t nbr[6];
};

// Relaxation solver states.
enum {
    RS_NEWTON = 0,
    RS_NEWTON_LAST = 1,  // one more evaluation after a step below tol_step
    RS_BIS_INIT = 2,     // evaluate both bracket ends
    RS_BIS = 3,
    RS_DONE = 4,
    RS_FALLBACK = 5,
    RS_EVAL1 = 6         // one evaluation at gamma = 1 (bookkeeping of non-relaxed steps)
};

// Per-case state of the step (device resident, persists across steps).
struct CaseState {
    double dt;
    double gamma;       // current evaluation point
    double gamma_b;     // second evaluation point (bracket end)
    double gamma_prev;  // accepted gamma of the previous step
    double gamma_acc;   // accepted gamma of this step
    double dH;
    double r, rp;       // residual and derivative at the last evaluation
    double lo, hi;      // bisection bracket
    double offset;      // H(U_n) - H(U_0) (initial anchoring)
    double H_delta;     // H(U_{n+1}) - H(U_n) at the accepted gamma
    double e[PERRK_MAXB];  // stage entropy production of the b_i != 0 stages
    double t;           // accumulated relaxed time
    double ghist[3];    // last three accepted gamma - 1, most recent first (learned guess features)
    int32_t state, k, iters, passes, flags, bis_count, widen, trivial;
    int32_t nsteps;     // steps taken (the learned guess needs three earlier gammas)
    int32_t pad_;
};

struct RelaxParams {
    double tol_r, tol_step, bis_lo, bis_hi;
    int32_t max_newton, max_bisect, anchor, relax;
    int32_t guess;
    int32_t nb;          // number of b != 0 stages (entropy-production slots, in stage order)
    int32_t nb_pre;      // those before the last stage (their sums are known before it runs)
    double bw[PERRK_MAXB];  // their weights
};

// Arguments of one stage launch.  The per-level coefficients of the stage live
// in device memory: coef[r] multiplies K_1, coef[PERRK_MAXR + r] multiplies K_{i-1}.
struct StageArgs {
    const double *U;          // U_n (caller state)
    const float *U32;         // U_n rounded to single precision (read by single-precision stages after the first)
    float *U32_out;           // first stage: writes that copy (every element runs the first stage), or NULL
    const void *K1;           // K_1 (stage storage type)
    const void *Kp;           // K_{i-1}
    void *Kout;               // K_i (stage storage type); unused for the last stage
    double *d_out;            // last stage: d = b_1 K_1 + b_{S-1} K_{S-1} + b_S K_S
    const ElemInfo *elem;
    const ActiveEntry *active; // active elements of the stage
    int32_t n_active;
    const CaseState *cs;      // dt per case
    double *ep_partial;       // [nelem] per-element J sum q w.K, or NULL
    int32_t *err;             // bit 1: non-physical, bit 2: non-finite state formed
    int64_t nelem;
    double gam, gm1, inv_gm1; // gamma, gamma - 1, 1 / (gamma - 1)
    int32_t flux;             // surface flux (PERRK_FLUX_*)
    int32_t volume;           // volume term (PERRK_VOLUME_*)
    int32_t sys;              // PERRK_SYSTEM_*
    double c_h;               // GLM-MHD divergence-cleaning speed
    int32_t viscous;          // 1: Navier-Stokes-Fourier terms (BR1), 2D double precision
    double mu, prandtl;       //   viscosity and Prandtl number
    double *grad;             //   [8][nelem][node] gradients of (rho, v_x, v_y, T) (d then q)
    const ActiveEntry *active_all;  // every element (the gradient pass)
    int32_t n_all;
    double c_stage;           //   c_i of the stage (boundary values at t_n + c_i dt)
    double x_lo, x_hi;        //   x ends of the viscous-shock mesh (its boundaries)
    double b1, bsm1, bs;      // last stage weights
    double b_acc;             // stages with b_i != 0 other than 1, S-1, S: b_i (K_i enters d here)
    int32_t acc_mode;         //   1: d = b_i K_i, 2: d += b_i K_i, 0: no contribution
    int32_t d_has;            // last stage: d already holds the contributions of such stages
    double *k64_out;          // optional double copy of K_i (b_i != 0 stages in mixed precision)
    const double *k64_1;      // last stage: double copies of K_1 and K_{S-1}, or NULL to read the
    const double *k64_sm1;    //   stage storage
    double *rx_partial;       // last stage: [nelem][4] partials of the first residual evaluation
                              //   at each case's gamma (as a residual pass writes them), or NULL
};

// Stage kernel variants.
enum { SK_FIRST = 0, SK_MID = 1, SK_LAST = 2 };

struct LaunchCfg {
    int epb_mult;   // wavefronts (of 64 lanes) per workgroup (1, 2, 4 or 8)
    int one_dir;    // Euler stages with the EC fluxes: 1 = the directions' pairs and faces one
                    // direction at a time (smaller LDS slot), 0 = the two-direction phases
};
#define PERRK_MAX_WPB 8

// Workgroup LDS bytes of a stage launch with wpb wavefronts per workgroup
// (sys: PERRK_SYSTEM_*, or 2 for the Navier-Stokes stage kernel; one_dir: the
// one-direction-at-a-time slots of the stages with the EC fluxes).
size_t stage_lds_bytes(int dim, int variant, int wpb, int sys, bool one_dir);

// Kernel launchers (perrk_kernels.hip).
// variant: 0 double flux / double storage, 1 float / float, 2 double flux / float storage;
// flux = 0 with a.volume = 0 runs the EC-only kernel, anything else the kernel with
// run-time selected surface flux and volume term; a.sys = 1 runs the GLM-MHD
// kernel (2D, variant 0 only); a.viscous = 1 runs the BR1 gradient pass and the
// Navier-Stokes stage kernel (2D, variant 0 only).  sys: PERRK_SYSTEM_*.
hipError_t launch_stage(int dim, int variant, int flux, int kind, const StageArgs &a, const double *coef,
                        LaunchCfg cfg, hipStream_t s);
// phase 0: after the last stage, everything below; 1: before the last stage (the
// entropy production of the earlier stages, solver reset, starting gamma); 2: after
// a last stage that evaluated the first residual (its entropy production, dH, and
// the solver update from that evaluation).  Cases of more than PERRK_RED_CHUNK
// elements are summed in chunks first (ch; none when n_chunks = 0).
#define PERRK_RED_CHUNK 8192  // elements per chunk of a large case's sums (fixed: results depend on it)
struct PrepChunks {
    int n_chunks = 0;                // chunks over all cases of more than PERRK_RED_CHUNK elements
    const int64_t *range = nullptr;  // [n_chunks][2]: first and end element of each chunk
    const int32_t *case_chunk = nullptr;  // [n_cases + 1]: case c's chunks [case_chunk[c], case_chunk[c+1])
    double *sums = nullptr;          // [n_chunks][PERRK_MAXB + 4]
};
hipError_t launch_relax_prepare(CaseState *cs, const int64_t *case_off, int n_cases,
                                const double *ep_partial, int64_t nelem, RelaxParams rp,
                                const float *mlp, int phase, const double *rx_partial, const PrepChunks &ch,
                                int32_t *live, hipStream_t s);
// live: one word per launched residual pass of a step, cleared when the step
// begins (the prepare kernel raises the first pass's word, the finalize after
// pass p that of pass p + 1; a pass and its finalize leave at once while theirs
// is zero).
hipError_t launch_relax_pass(int dim, int sys, const double *U, const double *d, const ElemInfo *elem,
                             const CaseState *cs, double *partial, int64_t nelem, double gam, bool first,
                             const int32_t *live, hipStream_t s);
hipError_t launch_relax_finalize(CaseState *cs, const int64_t *case_off, int n_cases,
                                 const double *partial, RelaxParams rp, const int32_t *live_in,
                                 int32_t *live_out, hipStream_t s);
hipError_t launch_relax_complete(int dim, int sys, const double *U, const double *d, const ElemInfo *elem,
                                 CaseState *cs, const int64_t *case_off, int n_cases,
                                 double *partial, int64_t nelem, double gam, RelaxParams rp,
                                 const int32_t *err, hipStream_t s);
hipError_t launch_final_update(int dim, int sys, double *U, const double *d, const ElemInfo *elem,
                               const CaseState *cs, int32_t *err, int64_t nelem,
                               hipStream_t s);
hipError_t launch_entropy(int dim, int sys, const double *U, const ElemInfo *elem, double *partial,
                          double *H_out, const int64_t *case_off, int n_cases, int64_t nelem,
                          double gam, int32_t *err, hipStream_t s);
hipError_t launch_init_cases(CaseState *cs, int n_cases, hipStream_t s);
hipError_t launch_set_dt(CaseState *cs, const double *dt, int n_cases, hipStream_t s);
hipError_t launch_clear_err(int32_t *err, int n, hipStream_t s);  // err[0..n-1] = 0
// as a step begins: *err_step = 0 and live[0..n_live-1] = 0 (n_live <= 64)
hipError_t launch_clear_step(int32_t *err_step, int32_t *live, int n_live, hipStream_t s);
