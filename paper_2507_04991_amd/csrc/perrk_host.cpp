// perrk_host.cpp -- host side of libperrk: descriptor validation, element
// tables, per-stage active lists, buffer planning, the launch sequence of
// one P-ERRK step (optionally captured once into a hipGraph), and the C ABI
// declared in include/perrk.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "perrk.h"
#include "perrk_internal.h"

struct perrk_ctx {
    std::string err;
    // problem
    int dim = 2, V = 4, npe = 16, n_cases = 1, precision = 0, flux = 0, volume = 0, sys = 0;
    double c_h = 0.0;
    int viscous = 0, bc_x = 0;        // Navier-Stokes-Fourier terms; viscous-shock x boundaries
    double mu = 0.0, prandtl = 0.75, x_lo = 0.0, x_hi = 0.0;
    double *d_grad = nullptr;         // [8][nelem][node] BR1 gradients of the current stage
    double gam = 1.4;
    int64_t nelem = 0;
    std::vector<int64_t> case_off;
    // tableau
    int order = 2, S = 2, R = 1;
    std::vector<int> E;
    std::vector<double> c, b, a_sub;
    std::vector<int> bstages;  // stages with b_i != 0
    perrk_options opt{};
    RelaxParams rp{};
    LaunchCfg cfg{4, 0};            // default stage launch shape
    bool can_one_dir = false;       // Euler with the EC fluxes, GLM-MHD: stages may take one direction at a time
    std::vector<LaunchCfg> scfg;    // per stage (autotuned at the first step when opt.tune)
    bool tuned = false;
    std::string tune_report;
    size_t max_lds = 65536;         // LDS bytes a workgroup may use on this device
    std::vector<int32_t> n_active;  // per stage
    std::vector<int64_t> active_off;  // start of each stage's list in d_active
    // viscous terms: per stage, the elements whose gradients the stage reads (its
    // active elements and their face neighbours), a list in d_active as well
    std::vector<int32_t> n_grad;
    std::vector<int64_t> grad_off;
    std::vector<std::vector<int64_t>> grad_per_level;
    std::vector<ElemInfo> h_elem;  // element table (host copy)
    std::vector<int32_t> h_dims;   // [n_cases][3] elements per direction
    int tile = 1;                  // element tile of the active lists (1..PERRK_TILES)
    size_t n_list = 0;             // entries in d_active
    // streams and events
    hipStream_t user_stream = nullptr, stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // device buffers
    ElemInfo *d_elem = nullptr;
    ActiveEntry *d_active = nullptr;  // per stage: active elements with their neighbour words
    int64_t *d_case_off = nullptr;
    // chunks of the per-case sums of cases of more than PERRK_RED_CHUNK elements
    PrepChunks chunks;
    int64_t *d_chunk_range = nullptr;
    int32_t *d_case_chunk = nullptr;
    double *d_chunk_sums = nullptr;
    CaseState *d_cs = nullptr;
    double *d_coef = nullptr;  // [S][2 * PERRK_MAXR]
    void *d_K1 = nullptr, *d_Ka = nullptr, *d_Kb = nullptr;
    double *d_k64_1 = nullptr, *d_k64_sm1 = nullptr;  // mixed: double copies of K_1 / K_{S-1} when b != 0
    float *d_U32 = nullptr;  // mixed modes: U_n rounded to single precision (written by the first stage)
    double *d_d = nullptr, *d_ep = nullptr, *d_partial = nullptr, *d_H = nullptr, *d_dt = nullptr;
    int32_t *d_err = nullptr;
    int32_t *d_live = nullptr;  // per launched residual pass: some case still needs it (fast_passes + 1 words)
    float *d_mlp = nullptr;
    bool have_mlp = false;
    bool fused_first = false;  // the last stage evaluates the first relaxation residual
    // pinned host staging
    static constexpr int NRING = 8;
    double *h_dt = nullptr;  // [NRING][n_cases]
    hipEvent_t ring_ev[NRING] = {};
    int ring = 0;
    CaseState *h_cs = nullptr;
    int32_t *h_err = nullptr;
    double *h_H = nullptr;
    // profiling
    bool profiling = false;
    static constexpr int NEV = 192;
    hipEvent_t pev[NEV] = {};
    int npev = 0;
    int pcls[NEV / 2] = {};
    double pbytes[NEV / 2] = {};
    int pstage[NEV / 2] = {};
    perrk_kernel_stat stats[PERRK_K_CLASSES] = {};
    std::vector<perrk_kernel_stat> sstats;  // per stage
    std::vector<double> stage_bytes;  // algorithmic bytes of each stage launch
    double pass_bytes = 0.0, update_bytes = 0.0;
    // graph
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    void *graph_u = nullptr;
};

namespace {

int fail(perrk_ctx *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

#define HIPCHECK(ctx, call)                                                                     \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((ctx), PERRK_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

struct Checker {
    char *msg;
    size_t len;
    int bad(const char *fmt, ...)
    {
        if (msg && len) {
            va_list ap;
            va_start(ap, fmt);
            vsnprintf(msg, len, fmt, ap);
            va_end(ap);
        }
        return PERRK_EINVAL;
    }
};

// Dense Butcher matrix of level r (row i: c_i - a in column 0, a in column i-1).
std::vector<double> dense_A(const perrk_tableau_desc *t, int r)
{
    const int S = t->S;
    std::vector<double> A((size_t)S * S, 0.0);
    for (int i = 1; i < S; ++i) {
        const double a = t->a_sub[r * S + i];
        A[i * S + 0] += t->c[i] - a;
        A[i * S + i - 1] += a;
    }
    return A;
}

std::vector<double> matvec(const std::vector<double> &A, const std::vector<double> &x, int S)
{
    std::vector<double> y(S, 0.0);
    for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j) y[i] += A[i * S + j] * x[j];
    return y;
}

double dot(const double *b, const std::vector<double> &x)
{
    double s = 0.0;
    for (size_t i = 0; i < x.size(); ++i) s += b[i] * x[i];
    return s;
}

int validate(const perrk_mesh_desc *m, const perrk_partition_desc *p, const perrk_tableau_desc *t,
             const perrk_options *o, char *msg, size_t len)
{
    Checker ck{msg, len};
    if (msg && len) msg[0] = 0;
    if (!m || !p || !t) return ck.bad("null descriptor");
    if (m->dim != 2 && m->dim != 3) return ck.bad("dim must be 2 or 3 (got %d)", m->dim);
    if (m->n_cases < 1) return ck.bad("n_cases must be >= 1");
    if (!m->n_elem_dir || !m->face_coords) return ck.bad("null mesh arrays");
    if (!(m->gas_gamma > 1.0) || !std::isfinite(m->gas_gamma)) return ck.bad("gas_gamma must be > 1");
    if (m->system != PERRK_SYSTEM_EULER && m->system != PERRK_SYSTEM_GLM_MHD)
        return ck.bad("unknown system %d", m->system);
    if (m->viscous != 0 && m->viscous != 1) return ck.bad("viscous must be 0 or 1");
    if (m->viscous) {
        if (m->dim != 2 || m->system != PERRK_SYSTEM_EULER || m->precision != PERRK_FP64)
            return ck.bad("viscous terms need dim = 2, the Euler system and PERRK_FP64");
        if (!(m->mu >= 0.0) || !std::isfinite(m->mu) || !(m->prandtl > 0.0) || !std::isfinite(m->prandtl))
            return ck.bad("viscous terms need mu >= 0 and prandtl > 0");
    }
    if (m->bc_x != 0 && m->bc_x != 1) return ck.bad("bc_x must be 0 or 1");
    if (m->bc_x == 1 && (!m->viscous || m->n_cases != 1))
        return ck.bad("the viscous-shock boundaries need the viscous terms and one case");
    if (m->system == PERRK_SYSTEM_GLM_MHD) {
        if (m->dim != 2) return ck.bad("GLM-MHD needs dim = 2");
        if (m->precision != PERRK_FP64) return ck.bad("GLM-MHD runs in PERRK_FP64 only");
        if (m->surface_flux != PERRK_FLUX_EC && m->surface_flux != PERRK_FLUX_LLF &&
            m->surface_flux != PERRK_FLUX_CENTRAL)
            return ck.bad("GLM-MHD surface flux must be EC, LLF or CENTRAL (got %d)", m->surface_flux);
        if (!(m->glm_ch >= 0.0) || !std::isfinite(m->glm_ch)) return ck.bad("glm_ch must be finite and >= 0");
    } else if (m->surface_flux < PERRK_FLUX_EC || m->surface_flux > PERRK_FLUX_HLLC) {
        return ck.bad("unknown surface flux %d", m->surface_flux);
    }
    if (m->volume_integral != PERRK_VOLUME_FLUX_DIFFERENCING && m->volume_integral != PERRK_VOLUME_WEAK)
        return ck.bad("unknown volume integral %d", m->volume_integral);
    if (m->precision != PERRK_FP64 && m->precision != PERRK_MIXED && m->precision != PERRK_MIXED_ALL)
        return ck.bad("unknown precision %d", m->precision);
    int64_t total = 0;
    const double *f = m->face_coords;
    for (int c = 0; c < m->n_cases; ++c) {
        int64_t ne = 1;
        for (int d = 0; d < 3; ++d) {
            const int n = m->n_elem_dir[3 * c + d];
            if (d < m->dim) {
                if (n < 2 || n > (1 << 20)) return ck.bad("case %d: n[%d] = %d out of range", c, d, n);
                for (int k = 0; k < n; ++k)
                    if (!(f[k + 1] > f[k]) || !std::isfinite(f[k]) || !std::isfinite(f[k + 1]))
                        return ck.bad("case %d: face coordinates of direction %d not increasing", c, d);
                f += n + 1;
                ne *= n;
            } else if (n != 1) {
                return ck.bad("case %d: n[2] must be 1 in 2D", c);
            }
        }
        total += ne;
    }
    const int64_t npe = m->dim == 2 ? 16 : 64;
    if (!perrk_node_count_ok(total * npe))
        return ck.bad("too many nodes (%lld elements x %lld >= 2^29)", (long long)total, (long long)npe);
    const int S = t->S, R = t->n_levels;
    if (t->order < 2 || t->order > 4) return ck.bad("order must be 2, 3 or 4");
    if (S < 2 || S > PERRK_MAXS) return ck.bad("S must be in 2..%d", PERRK_MAXS);
    if (R < 1 || R > PERRK_MAXR) return ck.bad("n_levels must be in 1..%d", PERRK_MAXR);
    if (!t->E || !t->c || !t->b || !t->a_sub) return ck.bad("null tableau arrays");
    if (p->n_levels != R) return ck.bad("partition has %d levels, tableau %d", p->n_levels, R);
    if (!p->elem_level) return ck.bad("null elem_level");
    for (int64_t e = 0; e < total; ++e)
        if (p->elem_level[e] < 0 || p->elem_level[e] >= R)
            return ck.bad("element %lld has level %d", (long long)e, p->elem_level[e]);
    if (t->c[0] != 0.0) return ck.bad("c_1 must be 0");
    for (int i = 0; i < S; ++i) {
        if (!std::isfinite(t->c[i]) || !std::isfinite(t->b[i])) return ck.bad("non-finite c or b");
        if (t->b[i] < 0.0) return ck.bad("b_%d < 0", i + 1);
    }
    {
        int nb = 0;
        for (int i = 0; i < S; ++i) nb += t->b[i] != 0.0;
        if (nb > PERRK_MAXB) return ck.bad("%d weights b_i != 0: at most %d", nb, PERRK_MAXB);
    }
    for (int r = 0; r < R; ++r) {
        const int E = t->E[r];
        if (E < 2 || E > S) return ck.bad("level %d: E = %d outside 2..S", r, E);
        for (int i = 0; i < S; ++i) {
            const double a = t->a_sub[r * S + i];
            if (!std::isfinite(a)) return ck.bad("non-finite a_sub");
            if (i <= 1 && a != 0.0) return ck.bad("level %d: a_sub[%d] must be 0", r, i);
            if (i >= 1 && i <= S - E + 1 && a != 0.0)
                return ck.bad("level %d: stage %d is skipped or first evaluated, a_{i,i-1} must be 0", r,
                              i + 1);
        }
        for (int i = 1; i < S; ++i)
            if (t->b[i] != 0.0 && i < S - E + 1)
                return ck.bad("b_%d != 0 needs every level to evaluate stage %d (level %d has E = %d)", i + 1,
                              i + 1, r, E);
    }
    // order conditions of the partitioned method for every level combination
    std::vector<double> one(S, 1.0), cv(t->c, t->c + S), c2(S), c3(S);
    for (int i = 0; i < S; ++i) {
        c2[i] = cv[i] * cv[i];
        c3[i] = c2[i] * cv[i];
    }
    const double tol = 1e-10;
    if (std::fabs(dot(t->b, one) - 1.0) > tol) return ck.bad("order 1 condition sum b = 1 violated");
    if (std::fabs(dot(t->b, cv) - 0.5) > tol) return ck.bad("order 2 condition b.c = 1/2 violated");
    std::vector<std::vector<double>> A(R);
    for (int r = 0; r < R; ++r) A[r] = dense_A(t, r);
    if (t->order >= 3) {
        if (std::fabs(dot(t->b, c2) - 1.0 / 3.0) > tol) return ck.bad("order 3: b.c^2 = 1/3 violated");
        for (int r = 0; r < R; ++r)
            if (std::fabs(dot(t->b, matvec(A[r], cv, S)) - 1.0 / 6.0) > tol)
                return ck.bad("order 3: b.A c = 1/6 violated for level %d", r);
    }
    if (t->order >= 4) {
        if (std::fabs(dot(t->b, c3) - 0.25) > tol) return ck.bad("order 4: b.c^3 = 1/4 violated");
        for (int r = 0; r < R; ++r) {
            std::vector<double> Ac = matvec(A[r], cv, S), cAc(S);
            for (int i = 0; i < S; ++i) cAc[i] = cv[i] * Ac[i];
            if (std::fabs(dot(t->b, cAc) - 0.125) > tol) return ck.bad("order 4: b.(c A c) = 1/8 (level %d)", r);
            if (std::fabs(dot(t->b, matvec(A[r], c2, S)) - 1.0 / 12.0) > tol)
                return ck.bad("order 4: b.A c^2 = 1/12 (level %d)", r);
            for (int s = 0; s < R; ++s)
                if (std::fabs(dot(t->b, matvec(A[r], matvec(A[s], cv, S), S)) - 1.0 / 24.0) > tol)
                    return ck.bad("order 4: b.A A c = 1/24 (levels %d, %d)", r, s);
        }
    }
    if (o) {
        if (o->max_newton < 0 || o->max_newton > 100) return ck.bad("max_newton out of range");
        if (o->max_bisect < 0 || o->max_bisect > 200) return ck.bad("max_bisect out of range");
        if (!(o->tol_r >= 0.0) || !(o->tol_step >= 0.0)) return ck.bad("tolerances must be >= 0");
        if (!(o->bisect_lo > 0.0 && o->bisect_lo < 1.0 && o->bisect_hi > 1.0))
            return ck.bad("bracket must satisfy 0 < lo < 1 < hi");
        if (o->anchor != PERRK_ANCHOR_STEP && o->anchor != PERRK_ANCHOR_INITIAL) return ck.bad("bad anchor");
        if (o->guess != PERRK_GUESS_PREV && o->guess != PERRK_GUESS_MLP && o->guess != PERRK_GUESS_EXTRAP)
            return ck.bad("bad guess");
        if (o->fast_passes < 1 || o->fast_passes > 16) return ck.bad("fast_passes must be in 1..16");
        if (o->tune != 0 && o->tune != 1 && o->tune != -1 && o->tune != -2 && o->tune != -4 && o->tune != -8)
            return ck.bad("tune must be 1, 0, -1, -2, -4 or -8");
        if (o->tile < 0 || o->tile > PERRK_TILES) return ck.bad("tile must be in 0..%d", PERRK_TILES);
        if (o->phases < 0 || o->phases > 2) return ck.bad("phases must be 0, 1 or 2");
    }
    return PERRK_OK;
}

void free_all(perrk_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    void *dev[] = {c->d_elem, c->d_active, c->d_case_off, c->d_cs, c->d_coef, c->d_K1, c->d_Ka,
                   c->d_Kb, c->d_d, c->d_ep, c->d_partial, c->d_H, c->d_dt, c->d_err, c->d_mlp,
                   c->d_k64_1, c->d_k64_sm1, c->d_grad, c->d_U32, c->d_chunk_range, c->d_case_chunk,
                   c->d_chunk_sums, c->d_live};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    void *host[] = {c->h_dt, c->h_cs, c->h_err, c->h_H};
    for (void *p : host)
        if (p) (void)hipHostFree(p);
    for (auto &e : c->ring_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->pev)
        if (e) (void)hipEventDestroy(e);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    if (c->stream) (void)hipStreamDestroy(c->stream);
}

// Profiling: events around one launch.
hipError_t mark_begin(perrk_ctx *c)
{
    if (!c->profiling || c->npev + 2 > perrk_ctx::NEV) return hipSuccess;
    return hipEventRecord(c->pev[c->npev], c->stream);
}

hipError_t mark_end(perrk_ctx *c, int cls, double bytes, int stage = -1)
{
    if (!c->profiling || c->npev + 2 > perrk_ctx::NEV) return hipSuccess;
    const hipError_t e = hipEventRecord(c->pev[c->npev + 1], c->stream);
    c->pcls[c->npev / 2] = cls;
    c->pstage[c->npev / 2] = stage;
    c->pbytes[c->npev / 2] = bytes;
    c->npev += 2;
    return e;
}

// Element tiles the active lists keep together (option `tile`, 1..PERRK_TILES).
// 2D: tiles of 32 quadrilaterals, the elements of a full workgroup of
// PERRK_MAX_WPB wavefronts (4 quadrilaterals each), 8 x 4, 4 x 8, 16 x 2 or 32 x 1,
// row by row inside a tile.  3D: cubes of 8^3, 4^3 or 16^3 hexahedra (x fastest
// inside a cube), or whole rows (x fastest).
constexpr int TILE_2D[PERRK_TILES][2] = {{8, 4}, {4, 8}, {16, 2}, {32, 1}};
constexpr int TILE_3D[PERRK_TILES] = {8, 4, 16, 0};

const char *tile_name(int dim, int tile)
{
    static const char *const n2[PERRK_TILES] = {"8x4", "4x8", "16x2", "32x1"};
    static const char *const n3[PERRK_TILES] = {"8^3", "4^3", "16^3", "rows"};
    return dim == 2 ? n2[tile - 1] : n3[tile - 1];
}

// Active element list of every stage (stage i evaluates the levels with
// E >= S - i + 1, 0-based; stage 1 every element) in the element order of the
// tile choice, and with viscous terms the gradient lists; fills n_active,
// active_off (and n_grad, grad_off, grad_per_level).  The lists' sizes do not
// depend on the tile.  In 2D, nbr[5], which 2D meshes do not need, records for
// each face f (bits 6f .. 6f + 5) the neighbour's position in the same list
// relative to the entry's, as offset + 31 for offsets in [-31, 31] and 63
// otherwise: the stage kernel takes the stage state of a neighbour that sits in
// its own workgroup from LDS.
void build_lists(perrk_ctx *c, int tile, std::vector<ActiveEntry> &order)
{
    const std::vector<ElemInfo> &elem = c->h_elem;
    std::vector<int64_t> visit;
    visit.reserve((size_t)c->nelem);
    for (int cs = 0; cs < c->n_cases; ++cs) {
        const int64_t base = c->case_off[cs];
        const int n0 = c->h_dims[3 * cs], n1 = c->h_dims[3 * cs + 1];
        if (c->dim == 3) {
            const int n2 = c->h_dims[3 * cs + 2];
            const int q = TILE_3D[tile - 1] > 0 ? TILE_3D[tile - 1] : std::max(n0, std::max(n1, n2));
            for (int tz = 0; tz < n2; tz += q)
                for (int ty = 0; ty < n1; ty += q)
                    for (int tx = 0; tx < n0; tx += q)
                        for (int iz = tz; iz < std::min(tz + q, n2); ++iz)
                            for (int iy = ty; iy < std::min(ty + q, n1); ++iy)
                                for (int ix = tx; ix < std::min(tx + q, n0); ++ix)
                                    visit.push_back(base + ix + (int64_t)n0 * (iy + (int64_t)n1 * iz));
            continue;
        }
        const int qx = TILE_2D[tile - 1][0], qy = TILE_2D[tile - 1][1];
        for (int ty = 0; ty < n1; ty += qy)
            for (int tx = 0; tx < n0; tx += qx)
                for (int iy = ty; iy < std::min(ty + qy, n1); ++iy)
                    for (int ix = tx; ix < std::min(tx + qx, n0); ++ix)
                        visit.push_back(base + ix + (int64_t)n0 * iy);
    }
    order.clear();
    std::vector<int64_t> pos((size_t)c->nelem, -1);  // list position of each element in the current stage
    c->n_active.assign(c->S, 0);
    c->active_off.assign(c->S + 1, 0);
    for (int i = 0; i < c->S; ++i) {
        c->active_off[i] = (int64_t)order.size();
        for (const int64_t e : visit) {
            const int E = c->E[elem[e].level];
            if (i == 0 || i >= c->S - E + 1) {
                ActiveEntry en{};
                en.elem_level = (int32_t)((uint32_t)e | ((uint32_t)elem[e].level << PERRK_NBR_SHIFT));
                en.case_id = elem[e].case_id;
                for (int k = 0; k < 6; ++k) en.nbr[k] = elem[e].nbr[k];
                if (c->dim == 2) {
                    // 2D meshes have no z neighbours: that word holds the boundary flags of the
                    // viscous-shock set-up (bit 0: left x face, bit 1: right x face)
                    const int ix = (int)(e % c->h_dims[0]);
                    en.nbr[4] = c->bc_x ? ((ix == 0 ? 1 : 0) | (ix == c->h_dims[0] - 1 ? 2 : 0)) : 0;
                    en.nbr[5] = 0;
                }
                pos[(size_t)e] = (int64_t)order.size() - c->active_off[i];
                order.push_back(en);
            }
        }
        c->n_active[i] = (int32_t)(order.size() - c->active_off[i]);
        if (c->dim == 2) {
            for (int64_t j = 0; j < c->n_active[i]; ++j) {
                ActiveEntry &en = order[(size_t)(c->active_off[i] + j)];
                uint32_t code = 0;
                for (int f = 0; f < 4; ++f) {
                    const int64_t q = pos[(size_t)((uint32_t)en.nbr[f] & PERRK_NBR_MASK)];
                    const int64_t off = q - j;
                    const uint32_t cf = (q >= 0 && off >= -31 && off <= 31) ? (uint32_t)(off + 31) : 63u;
                    code |= cf << (6 * f);
                }
                en.nbr[5] = (int32_t)code;
            }
        }
        for (int64_t j = 0; j < c->n_active[i]; ++j)
            pos[(size_t)((uint32_t)order[(size_t)(c->active_off[i] + j)].elem_level & PERRK_NBR_MASK)] = -1;
    }
    c->active_off[c->S] = (int64_t)order.size();
    if (c->viscous) {
        // BR1 needs the gradients at the nodes of a stage's active elements and at the
        // face nodes of their neighbours: the gradient pass of stage i runs over the
        // active elements and their face neighbours (in the first stage's order)
        c->n_grad.assign(c->S, 0);
        c->grad_off.assign(c->S, 0);
        c->grad_per_level.assign(c->S, std::vector<int64_t>(c->R, 0));
        std::vector<char> need((size_t)c->nelem);
        for (int i = 0; i < c->S; ++i) {
            std::fill(need.begin(), need.end(), 0);
            for (int64_t j = 0; j < c->n_active[i]; ++j) {
                const ActiveEntry &en = order[(size_t)(c->active_off[i] + j)];
                need[(size_t)((uint32_t)en.elem_level & PERRK_NBR_MASK)] = 1;
                for (int f = 0; f < 2 * c->dim; ++f)
                    need[(size_t)((uint32_t)elem[(uint32_t)en.elem_level & PERRK_NBR_MASK].nbr[f] & PERRK_NBR_MASK)] = 1;
            }
            c->grad_off[i] = (int64_t)order.size();
            for (int64_t j = 0; j < c->n_active[0]; ++j) {
                ActiveEntry en = order[(size_t)(c->active_off[0] + j)];
                const int64_t e = (uint32_t)en.elem_level & PERRK_NBR_MASK;
                if (!need[(size_t)e]) continue;
                en.nbr[5] = 0;
                order.push_back(en);
                c->grad_per_level[i][elem[e].level]++;
            }
            c->n_grad[i] = (int32_t)(order.size() - c->grad_off[i]);
        }
    }
}

// Arguments, kernel variant and kind of stage i.
void stage_setup(perrk_ctx *c, double *u, int i, StageArgs &a, int &variant, int &kind)
{
    a = StageArgs{};
    a.U = u;
    a.U32 = c->d_U32;
    a.U32_out = i == 0 ? c->d_U32 : nullptr;
    a.elem = c->d_elem;
    a.cs = c->d_cs;
    a.err = c->d_err + ERR_STEP;
    a.nelem = c->nelem;
    a.gam = c->gam;
    a.gm1 = c->gam - 1.0;
    a.inv_gm1 = 1.0 / (c->gam - 1.0);
    a.flux = c->flux;
    a.volume = c->volume;
    a.sys = c->sys;
    a.c_h = c->c_h;
    a.viscous = c->viscous;
    a.mu = c->mu;
    a.prandtl = c->prandtl;
    a.grad = c->d_grad;
    a.active_all = c->d_active;  // the first stage's list holds every element
    a.n_all = (int32_t)c->nelem;
    if (c->viscous) {  // the gradient pass: the stage's active elements and their neighbours
        a.active_all = c->d_active + c->grad_off[i];
        a.n_all = c->n_grad[i];
    }
    a.c_stage = c->c[i];
    a.x_lo = c->x_lo;
    a.x_hi = c->x_hi;
    const int S = c->S;
    void *kbuf[2] = {c->d_Ka, c->d_Kb};
    kind = i == 0 ? SK_FIRST : (i == S - 1 ? SK_LAST : SK_MID);
    a.K1 = c->d_K1;
    a.Kp = i >= 2 ? kbuf[(i - 2) % 2] : c->d_K1;
    a.Kout = i == 0 ? c->d_K1 : kbuf[(i - 1) % 2];
    a.d_out = c->d_d;
    a.active = c->d_active + c->active_off[i];
    a.n_active = c->n_active[i];
    a.b1 = c->b[0];
    a.bsm1 = (S >= 3) ? c->b[S - 2] : 0.0;
    a.bs = c->b[S - 1];
    // stages with b_i != 0 other than 1, S-1, S add b_i K_i to d as they finish
    // (the first of them writes d); the last stage then adds its terms to d
    bool any_acc = false;
    for (int j = 1; j < S - 2; ++j) {
        if (c->b[j] == 0.0) continue;
        if (j == i) {
            a.b_acc = c->b[j];
            a.acc_mode = any_acc ? 2 : 1;
        }
        any_acc = true;
    }
    if (i == S - 1) a.d_has = any_acc ? 1 : 0;
    a.ep_partial = nullptr;
    for (size_t j = 0; j < c->bstages.size(); ++j)
        if (c->bstages[j] == i) a.ep_partial = c->d_ep + j * (size_t)c->nelem;
    a.rx_partial = (kind == SK_LAST && c->fused_first) ? c->d_partial : nullptr;
    // MIXED: stages entering d and dH are evaluated in double precision
    const bool mixed = c->precision == PERRK_MIXED;
    variant = c->precision == PERRK_FP64 ? 0 : (mixed && c->b[i] != 0.0 ? 2 : 1);
    if (mixed && i == 0 && c->b[0] != 0.0 && S > 1) a.k64_out = c->d_k64_1;
    if (mixed && S >= 3 && i == S - 2 && c->b[S - 2] != 0.0) a.k64_out = c->d_k64_sm1;
    if (mixed && kind == SK_LAST) {
        a.k64_1 = c->b[0] != 0.0 ? c->d_k64_1 : nullptr;
        a.k64_sm1 = (S >= 3 && c->b[S - 2] != 0.0) ? c->d_k64_sm1 : nullptr;
    }
}

const double *stage_coef(const perrk_ctx *c, int i) { return c->d_coef + (size_t)i * 2 * PERRK_MAXR; }

// Rebuilds the active lists for element tile `tile` and uploads them (same size
// for every tile).
int use_tile(perrk_ctx *c, int tile)
{
    std::vector<ActiveEntry> order;
    build_lists(c, tile, order);
    if (order.size() != c->n_list) return fail(c, PERRK_EHIP, "internal: list size changed with the tile");
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipMemcpy(c->d_active, order.data(), sizeof(ActiveEntry) * order.size(), hipMemcpyHostToDevice));
    c->tile = tile;
    return PERRK_OK;
}

// Picks the wavefronts per workgroup of every stage launch, for Euler with the
// EC fluxes (option phases = 0) whether a stage with double-precision
// fluxes takes the two directions in one phase or one at a time (single-
// precision stages keep one phase: the selects cost them more than the smaller
// slot gains), and (option tile = 0) the element tile of the active lists, by
// timing the candidates on the caller's state: for each tile, every stage in
// step order with 1, 2, 4 and 8 wavefronts per workgroup in each phase
// structure (a stage launch only reads U_n and earlier stage registers, so
// repeating it is harmless); the tile with the smallest sum of its stages'
// best times is kept, with those launch shapes.  Each timed launch follows what
// precedes it in a step, so that it meets the caches of a step: the previous
// stage (with its chosen shape), or for stage 1 the other stages of a step
// (which also move stage 1's own outputs out of the caches, as a step does).
// Results do not depend on the tile, the phase structure or the launch shape.
int autotune(perrk_ctx *c, double *u)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHECK(c, hipEventCreate(&e0));
    HIPCHECK(c, hipEventCreate(&e1));
    const int first_tile = c->opt.tile > 0 ? c->opt.tile : 1;
    const int last_tile = c->opt.tile > 0 ? c->opt.tile : PERRK_TILES;
    std::string rep;
    int status = PERRK_OK, best_tile = c->tile;
    double best_sum = 1e300;
    std::vector<LaunchCfg> best_cfg = c->scfg;
    const int od_first = c->can_one_dir && c->opt.phases == 0 ? 0 : c->cfg.one_dir;
    const int od_last = c->can_one_dir && c->opt.phases == 0 ? 1 : c->cfg.one_dir;
    for (int tile = first_tile; tile <= last_tile && status == PERRK_OK; ++tile) {
        if (tile != c->tile && (status = use_tile(c, tile)) != PERRK_OK) break;
        std::vector<LaunchCfg> cfg = c->scfg;
        double sum = 0.0;
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "tile %s: waves per workgroup (stage: ms per candidate 1/2/4/8%s -> choice):",
                      tile_name(c->dim, tile), od_last > od_first ? ", then the same one direction at a time" : "");
        std::string tline = buf;
        for (int i = 0; i < c->S && status == PERRK_OK; ++i) {
            StageArgs a, ap;
            int variant = 0, kind = 0, variant_p = 0, kind_p = 0;
            stage_setup(c, u, i, a, variant, kind);
            if (i > 0) stage_setup(c, u, i - 1, ap, variant_p, kind_p);
            // the launches that precede stage i in a step
            auto context = [&]() -> hipError_t {
                if (i > 0)
                    return launch_stage(c->dim, variant_p, c->flux, kind_p, ap, stage_coef(c, i - 1), cfg[i - 1],
                                        c->stream);
                for (int j = 1; j < c->S; ++j) {
                    StageArgs aj;
                    int vj = 0, kj = 0;
                    stage_setup(c, u, j, aj, vj, kj);
                    const hipError_t e = launch_stage(c->dim, vj, c->flux, kj, aj, stage_coef(c, j), c->cfg, c->stream);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            };
            LaunchCfg best = c->cfg;
            float best_ms = 1e30f;
            std::snprintf(buf, sizeof buf, " %d:", i + 1);
            std::string line = buf;
            const int od_top = variant == 1 ? od_first : od_last;  // (variant 1: single-precision fluxes)
            for (int cand = 0; cand < 4 * (od_top - od_first + 1) && status == PERRK_OK; ++cand) {
                const LaunchCfg cf{1 << (cand & 3), od_first + (cand >> 2)};
                if (stage_lds_bytes(c->dim, variant, cf.epb_mult, c->viscous ? 2 : c->sys, cf.one_dir != 0) >
                    c->max_lds) {
                    line += " -";
                    continue;
                }
                if (launch_stage(c->dim, variant, c->flux, kind, a, stage_coef(c, i), cf, c->stream) != hipSuccess) {
                    (void)hipGetLastError();
                    line += " x";
                    continue;
                }
                float tmin = 1e30f;
                for (int r = 0; r < 3; ++r) {
                    if (context() != hipSuccess || hipEventRecord(e0, c->stream) != hipSuccess ||
                        launch_stage(c->dim, variant, c->flux, kind, a, stage_coef(c, i), cf, c->stream) != hipSuccess ||
                        hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                        status = fail(c, PERRK_EHIP, "autotuning launch failed: %s",
                                      hipGetErrorString(hipGetLastError()));
                        break;
                    }
                    float ms = 0.0f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    tmin = std::min(tmin, ms);
                }
                if (status != PERRK_OK) break;
                std::snprintf(buf, sizeof buf, " %.4f", tmin);
                line += buf;
                if (tmin < best_ms) {
                    best_ms = tmin;
                    best = cf;
                }
            }
            cfg[i] = best;
            sum += best_ms;
            std::snprintf(buf, sizeof buf, " -> %d%s;", best.epb_mult, best.one_dir ? " one direction at a time" : "");
            tline += line + buf;
        }
        std::snprintf(buf, sizeof buf, " sum %.4f ms. ", sum);
        rep += tline + buf;
        if (status == PERRK_OK && sum < best_sum) {
            best_sum = sum;
            best_tile = tile;
            best_cfg = cfg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != PERRK_OK) return status;
    if (best_tile != c->tile && (status = use_tile(c, best_tile)) != PERRK_OK) return status;
    c->scfg = best_cfg;
    c->tune_report = std::string("Chosen: tile ") + tile_name(c->dim, best_tile) + ". Autotuned: " + rep;
    c->tuned = true;
    return PERRK_OK;
}

// Enqueues one full step on ctx->stream (no host synchronisation).  With the
// Euler stage kernel, the solver is prepared before the last stage, whose epilogue
// evaluates the first residual at each case's starting gamma; otherwise the
// solver is prepared after the last stage and the first residual pass does it.
int enqueue_step(perrk_ctx *c, double *u)
{
    HIPCHECK(c, launch_clear_step(c->d_err + ERR_STEP, c->d_live, c->opt.fast_passes + 1, c->stream));
    const float *mlp = c->have_mlp ? c->d_mlp : nullptr;
    for (int i = 0; i < c->S; ++i) {
        StageArgs a;
        int variant = 0, kind = 0;
        stage_setup(c, u, i, a, variant, kind);
        if (kind == SK_LAST && c->fused_first) {
            HIPCHECK(c, mark_begin(c));
            HIPCHECK(c, launch_relax_prepare(c->d_cs, c->d_case_off, c->n_cases, c->d_ep, c->nelem, c->rp, mlp, 1,
                                             nullptr, c->chunks, nullptr, c->stream));
            HIPCHECK(c, mark_end(c, PERRK_K_SOLVER, 0.0));
        }
        HIPCHECK(c, mark_begin(c));
        HIPCHECK(c, launch_stage(c->dim, variant, c->flux, kind, a, stage_coef(c, i), c->scfg[i], c->stream));
        HIPCHECK(c, mark_end(c, kind == SK_FIRST ? PERRK_K_STAGE_FIRST
                                : (kind == SK_MID ? PERRK_K_STAGE_MID : PERRK_K_STAGE_LAST),
                             c->stage_bytes[i], i));
    }
    HIPCHECK(c, mark_begin(c));
    const int p0 = c->fused_first ? 1 : 0;  // the first launched pass
    HIPCHECK(c, launch_relax_prepare(c->d_cs, c->d_case_off, c->n_cases, c->d_ep, c->nelem, c->rp, mlp,
                                     c->fused_first ? 2 : 0, c->d_partial, c->chunks, c->d_live + p0, c->stream));
    HIPCHECK(c, mark_end(c, PERRK_K_SOLVER, 0.0));
    if (c->rp.relax) {
        // launched residual passes: fast_passes evaluations in all, the fused one included
        for (int p = p0; p < c->opt.fast_passes; ++p) {
            HIPCHECK(c, mark_begin(c));
            HIPCHECK(c, launch_relax_pass(c->dim, c->sys, u, c->d_d, c->d_elem, c->d_cs, c->d_partial, c->nelem, c->gam,
                                          p == 0, c->d_live + p, c->stream));
            HIPCHECK(c, mark_end(c, PERRK_K_RESIDUAL, c->pass_bytes));
            HIPCHECK(c, mark_begin(c));
            HIPCHECK(c, launch_relax_finalize(c->d_cs, c->d_case_off, c->n_cases, c->d_partial, c->rp,
                                              c->d_live + p, c->d_live + p + 1, c->stream));
            HIPCHECK(c, mark_end(c, PERRK_K_SOLVER, 0.0));
        }
    }
    HIPCHECK(c, mark_begin(c));
    HIPCHECK(c, launch_relax_complete(c->dim, c->sys, u, c->d_d, c->d_elem, c->d_cs, c->d_case_off, c->n_cases,
                                      c->d_partial, c->nelem, c->gam, c->rp, c->d_err, c->stream));
    HIPCHECK(c, mark_end(c, PERRK_K_SOLVER, 0.0));
    HIPCHECK(c, mark_begin(c));
    HIPCHECK(c, launch_final_update(c->dim, c->sys, u, c->d_d, c->d_elem, c->d_cs, c->d_err, c->nelem, c->stream));
    HIPCHECK(c, mark_end(c, PERRK_K_UPDATE, c->update_bytes));
    return PERRK_OK;
}

}  // namespace

extern "C" {

void perrk_default_options(perrk_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->relax = 1;
    o->max_newton = 10;
    o->tol_r = 1e-12;
    o->tol_step = 1e-15;
    o->anchor = PERRK_ANCHOR_STEP;
    o->max_bisect = 60;
    o->bisect_lo = 0.8;
    o->bisect_hi = 1.2;
    o->guess = PERRK_GUESS_PREV;
    o->fast_passes = 3;
    o->use_graph = 1;
    o->tune = 1;
    o->tile = 0;
    o->phases = 0;
}

int perrk_validate(const perrk_mesh_desc *mesh, const perrk_partition_desc *part,
                   const perrk_tableau_desc *tab, const perrk_options *opts, char *msg, size_t msg_len)
{
    return validate(mesh, part, tab, opts, msg, msg_len);
}

int perrk_init(const perrk_mesh_desc *m, const perrk_partition_desc *p, const perrk_tableau_desc *t,
               const perrk_options *opts, void *stream, perrk_ctx **out)
{
    if (!out) return PERRK_EINVAL;
    *out = nullptr;
    perrk_options o;
    if (opts) o = *opts;
    else perrk_default_options(&o);
    char msg[512];
    const int st = validate(m, p, t, &o, msg, sizeof msg);
    if (st != PERRK_OK) {
        std::fprintf(stderr, "perrk_init: %s\n", msg);
        return st;
    }
    perrk_ctx *c = new (std::nothrow) perrk_ctx();
    if (!c) return PERRK_ENOMEM;
    c->opt = o;
    c->dim = m->dim;
    c->sys = m->system;
    c->viscous = m->viscous;
    c->mu = m->viscous ? m->mu : 0.0;
    c->prandtl = m->viscous ? m->prandtl : 0.75;
    c->bc_x = m->bc_x;
    if (m->bc_x) {
        c->x_lo = m->face_coords[0];
        c->x_hi = m->face_coords[m->n_elem_dir[0]];
    }
    c->c_h = m->system == PERRK_SYSTEM_GLM_MHD ? m->glm_ch : 0.0;
    c->V = m->system == PERRK_SYSTEM_GLM_MHD ? 9 : m->dim + 2;
    c->npe = m->dim == 2 ? 16 : 64;
    c->n_cases = m->n_cases;
    c->precision = m->precision;
    c->flux = m->surface_flux;
    c->volume = m->volume_integral;
    c->gam = m->gas_gamma;
    c->order = t->order;
    c->S = t->S;
    c->R = t->n_levels;
    c->E.assign(t->E, t->E + c->R);
    c->c.assign(t->c, t->c + c->S);
    c->b.assign(t->b, t->b + c->S);
    c->a_sub.assign(t->a_sub, t->a_sub + (size_t)c->R * c->S);
    for (int i = 0; i < c->S; ++i)
        if (c->b[i] != 0.0) c->bstages.push_back(i);

    // element tables (natural order, cases concatenated)
    std::vector<ElemInfo> elem;
    c->case_off.push_back(0);
    const double *f = m->face_coords;
    for (int cs = 0; cs < m->n_cases; ++cs) {
        const int n0 = m->n_elem_dir[3 * cs], n1 = m->n_elem_dir[3 * cs + 1];
        const int n2 = m->dim == 3 ? m->n_elem_dir[3 * cs + 2] : 1;
        const double *fx = f, *fy = fx + n0 + 1, *fz = fy + n1 + 1;
        f = fy + n1 + 1 + (m->dim == 3 ? n2 + 1 : 0);
        const int64_t base = c->case_off.back();
        for (int iz = 0; iz < n2; ++iz)
            for (int iy = 0; iy < n1; ++iy)
                for (int ix = 0; ix < n0; ++ix) {
                    ElemInfo ei{};
                    auto gid = [&](int x, int y, int z) {
                        return (int32_t)(base + x + (int64_t)n0 * (y + (int64_t)n1 * z));
                    };
                    ei.nbr[0] = gid((ix + n0 - 1) % n0, iy, iz);
                    ei.nbr[1] = gid((ix + 1) % n0, iy, iz);
                    ei.nbr[2] = gid(ix, (iy + n1 - 1) % n1, iz);
                    ei.nbr[3] = gid(ix, (iy + 1) % n1, iz);
                    ei.nbr[4] = m->dim == 3 ? gid(ix, iy, (iz + n2 - 1) % n2) : gid(ix, iy, iz);
                    ei.nbr[5] = m->dim == 3 ? gid(ix, iy, (iz + 1) % n2) : gid(ix, iy, iz);
                    const double hx = fx[ix + 1] - fx[ix], hy = fy[iy + 1] - fy[iy];
                    const double hz = m->dim == 3 ? fz[iz + 1] - fz[iz] : 2.0;
                    ei.metric[0] = 2.0 / hx;
                    ei.metric[1] = 2.0 / hy;
                    ei.metric[2] = 2.0 / hz;
                    ei.jac = 0.5 * hx * 0.5 * hy * (m->dim == 3 ? 0.5 * hz : 1.0);
                    const int64_t g = elem.size();
                    ei.level = p->elem_level[g];
                    ei.case_id = cs;
                    elem.push_back(ei);
                }
        c->case_off.push_back((int64_t)elem.size());
    }
    c->nelem = (int64_t)elem.size();
    // the neighbour's level travels with its index (element counts are below 2^28,
    // levels below 16), so a stage reads a neighbour's stage state without first
    // loading the neighbour's table entry
    for (auto &ei : elem)
        for (int k = 0; k < 6; ++k)
            ei.nbr[k] = (int32_t)((uint32_t)ei.nbr[k] | ((uint32_t)elem[ei.nbr[k]].level << PERRK_NBR_SHIFT));

    c->h_elem.swap(elem);  // kept: the autotuner rebuilds the lists for other tiles
    c->h_dims.assign(m->n_elem_dir, m->n_elem_dir + 3 * m->n_cases);
    c->tile = o.tile > 0 ? o.tile : 1;
    std::vector<ActiveEntry> order;
    build_lists(c, c->tile, order);
    c->n_list = order.size();
    // per-stage coefficients (without dt): K_1 and K_{i-1} multipliers per level
    std::vector<double> coef((size_t)c->S * 2 * PERRK_MAXR, 0.0);
    for (int i = 1; i < c->S; ++i)
        for (int r = 0; r < c->R; ++r) {
            const double a = (i >= 2) ? c->a_sub[(size_t)r * c->S + i] : 0.0;
            coef[(size_t)i * 2 * PERRK_MAXR + r] = c->c[i] - a;
            coef[(size_t)i * 2 * PERRK_MAXR + PERRK_MAXR + r] = a;
        }
    // relaxation parameters
    RelaxParams rp{};
    rp.tol_r = o.tol_r;
    rp.tol_step = o.tol_step;
    rp.bis_lo = o.bisect_lo;
    rp.bis_hi = o.bisect_hi;
    rp.max_newton = o.max_newton;
    rp.max_bisect = o.max_bisect;
    rp.anchor = o.anchor;
    rp.relax = o.relax;
    rp.guess = o.guess;
    rp.nb = (int)c->bstages.size();
    rp.nb_pre = 0;
    for (int j = 0; j < rp.nb && j < PERRK_MAXB; ++j) {
        rp.bw[j] = c->b[c->bstages[j]];
        if (c->bstages[j] < c->S - 1) rp.nb_pre = j + 1;
    }
    c->rp = rp;
    // the Euler stage kernel's last stage evaluates the first residual of the solve
    c->fused_first = c->sys == PERRK_SYSTEM_EULER && !c->viscous;
    // stages that may take the directions one at a time: Euler with the EC fluxes
    // (pairs and faces of a direction together), GLM-MHD with any fluxes (pairs only)
    c->can_one_dir = (c->fused_first && c->flux == PERRK_FLUX_EC && c->volume == PERRK_VOLUME_FLUX_DIFFERENCING) ||
                     c->sys == PERRK_SYSTEM_GLM_MHD;
    // GLM-MHD: 24 KB of LDS per wavefront (17 KB one direction at a time); Navier-Stokes: 19 KB
    c->cfg.epb_mult = c->sys == PERRK_SYSTEM_GLM_MHD ? 1 : (c->viscous ? 2 : 4);
    c->cfg.one_dir = c->can_one_dir && c->opt.phases == 2 ? 1 : 0;
    c->scfg.assign(c->S, c->cfg);
    c->sstats.assign(c->S, perrk_kernel_stat{});

    // algorithmic (compulsory) bytes of each launch
    {
        const double dofe = (double)c->V * c->npe;  // DOF per element
        const double kb = c->precision == PERRK_FP64 ? 8.0 : 4.0;
        std::vector<int64_t> per_level(c->R, 0);
        for (int64_t e = 0; e < c->nelem; ++e) per_level[c->h_elem[e].level]++;
        c->stage_bytes.assign(c->S, 0.0);
        int first_acc = -1;  // first stage with b_i != 0 other than 1, S-1, S
        for (int j = 1; j < c->S - 2 && first_acc < 0; ++j)
            if (c->b[j] != 0.0) first_acc = j;
        for (int i = 0; i < c->S; ++i) {
            double bytes = 0.0;
            for (int r = 0; r < c->R; ++r) {
                if (!(i == 0 || i >= c->S - c->E[r] + 1)) continue;
                const double c1 = coef[(size_t)i * 2 * PERRK_MAXR + r];
                const double cp = coef[(size_t)i * 2 * PERRK_MAXR + PERRK_MAXR + r];
                const bool mixed = c->precision == PERRK_MIXED;
                const bool last = (i == c->S - 1);
                // single-precision stages after the first read U_n in single precision;
                // the first stage writes that copy
                const bool f32 = c->precision == PERRK_MIXED_ALL || (mixed && c->b[i] == 0.0);
                double be = (i > 0 && i < c->S - 1 && f32) ? 4.0 : 8.0;  // U_n (double in the last stage)
                if (i == 0) {
                    if (c->precision != PERRK_FP64) be += 4.0;       // write its single-precision copy
                    be += kb;                                         // write K_1
                    if (mixed && c->b[0] != 0.0 && c->S > 1) be += 8.0;  // its double copy
                } else {
                    if (c1 != 0.0) be += kb;                          // K_1
                    if (cp != 0.0) be += kb;                          // K_{i-1}
                    if (last) {
                        be += 8.0;                                    // write d
                        if (first_acc >= 0) be += 8.0;                // read the accumulated d
                        if (c->S >= 3 && c->b[c->S - 2] != 0.0) be += mixed ? 8.0 : (cp != 0.0 ? 0.0 : kb);
                        if (c->b[0] != 0.0 && mixed) be += 8.0;       // double K_1 for d
                    } else {
                        be += kb;                                     // write K_i
                        if (mixed && i == c->S - 2 && c->b[i] != 0.0) be += 8.0;  // its double copy
                        if (i < c->S - 2 && c->b[i] != 0.0) be += first_acc == i ? 8.0 : 16.0;  // d
                    }
                }
                if (c->viscous) be += 16.0;  // the gradients of the node (8 doubles per 4 DOF)
                bytes += be * dofe * per_level[r];
            }
            if (c->viscous) {
                // the gradient pass over the stage's active elements and their neighbours:
                // its stage state and the gradient write
                for (int r = 0; r < c->R; ++r) {
                    const double c1 = coef[(size_t)i * 2 * PERRK_MAXR + r];
                    const double cp = coef[(size_t)i * 2 * PERRK_MAXR + PERRK_MAXR + r];
                    double be = 8.0 + 16.0;
                    if (i > 0 && c1 != 0.0) be += 8.0;
                    if (i > 0 && cp != 0.0) be += 8.0;
                    bytes += be * dofe * c->grad_per_level[i][r];
                }
            }
            c->stage_bytes[i] = bytes;
        }
        c->pass_bytes = 16.0 * dofe * c->nelem;
        c->update_bytes = 24.0 * dofe * c->nelem;
    }

    // device state
    const size_t M = (size_t)c->V * c->nelem * c->npe;
    const size_t ks = c->precision == PERRK_FP64 ? 8 : 4;
    auto bail = [&](int code) {
        free_all(c);
        delete c;
        return code;
    };
#define HIPINIT(call)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            std::fprintf(stderr, "perrk_init: %s failed: %s\n", #call, hipGetErrorString(e_)); \
            return bail(e_ == hipErrorOutOfMemory ? PERRK_ENOMEM : PERRK_EHIP);                 \
        }                                                                                       \
    } while (0)
    c->user_stream = (hipStream_t)stream;
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
            c->max_lds = (size_t)lds;
    }
    if (c->opt.tune < 0) {  // one given launch shape for every stage
        const int w = -c->opt.tune;
        if (stage_lds_bytes(c->dim, c->precision == PERRK_MIXED_ALL ? 1 : 0, w, c->viscous ? 2 : c->sys,
                            c->cfg.one_dir != 0) > c->max_lds) {
            std::fprintf(stderr, "perrk_init: %d wavefronts per workgroup need more LDS than the device has\n", w);
            return bail(PERRK_EINVAL);
        }
        c->cfg.epb_mult = w;
        c->scfg.assign(c->S, c->cfg);
    }
    HIPINIT(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIPINIT(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIPINIT(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    for (auto &e : c->ring_ev) HIPINIT(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPINIT(hipMalloc(&c->d_elem, sizeof(ElemInfo) * c->nelem));
    HIPINIT(hipMalloc(&c->d_active, sizeof(ActiveEntry) * order.size()));
    HIPINIT(hipMalloc(&c->d_case_off, sizeof(int64_t) * (c->n_cases + 1)));
    HIPINIT(hipMalloc(&c->d_cs, sizeof(CaseState) * c->n_cases));
    HIPINIT(hipMalloc(&c->d_coef, sizeof(double) * coef.size()));
    HIPINIT(hipMalloc(&c->d_K1, ks * M));
    HIPINIT(hipMalloc(&c->d_Ka, ks * M));
    HIPINIT(hipMalloc(&c->d_Kb, ks * M));
    HIPINIT(hipMalloc(&c->d_d, sizeof(double) * M));
    if (c->viscous) HIPINIT(hipMalloc(&c->d_grad, sizeof(double) * 8 * (size_t)c->nelem * c->npe));
    if (c->precision != PERRK_FP64) HIPINIT(hipMalloc(&c->d_U32, sizeof(float) * M));
    if (c->precision == PERRK_MIXED) {
        if (c->b[0] != 0.0) HIPINIT(hipMalloc(&c->d_k64_1, sizeof(double) * M));
        if (c->S >= 3 && c->b[c->S - 2] != 0.0) HIPINIT(hipMalloc(&c->d_k64_sm1, sizeof(double) * M));
    }
    HIPINIT(hipMalloc(&c->d_ep, sizeof(double) * std::max<size_t>(1, c->bstages.size()) * c->nelem));
    HIPINIT(hipMalloc(&c->d_partial, sizeof(double) * 4 * c->nelem));
    HIPINIT(hipMalloc(&c->d_H, sizeof(double) * c->n_cases));
    HIPINIT(hipMalloc(&c->d_dt, sizeof(double) * c->n_cases * perrk_ctx::NRING));
    HIPINIT(hipMalloc(&c->d_err, sizeof(int32_t) * ERR_WORDS));
    HIPINIT(hipMalloc(&c->d_live, sizeof(int32_t) * (16 + 1)));  // fast_passes <= 16
    HIPINIT(hipMalloc(&c->d_mlp, sizeof(float) * (PERRK_MLP_NW + 18)));
    HIPINIT(hipHostMalloc(&c->h_dt, sizeof(double) * c->n_cases * perrk_ctx::NRING, 0));
    HIPINIT(hipHostMalloc(&c->h_cs, sizeof(CaseState) * c->n_cases, 0));
    HIPINIT(hipHostMalloc(&c->h_err, sizeof(int32_t) * ERR_WORDS, 0));
    HIPINIT(hipHostMalloc(&c->h_H, sizeof(double) * c->n_cases, 0));
    HIPINIT(hipMemcpyAsync(c->d_elem, c->h_elem.data(), sizeof(ElemInfo) * c->nelem, hipMemcpyHostToDevice,
                           c->stream));
    HIPINIT(hipMemcpyAsync(c->d_active, order.data(), sizeof(ActiveEntry) * order.size(), hipMemcpyHostToDevice,
                           c->stream));
    HIPINIT(hipMemcpyAsync(c->d_case_off, c->case_off.data(), sizeof(int64_t) * (c->n_cases + 1),
                           hipMemcpyHostToDevice, c->stream));
    HIPINIT(hipMemcpyAsync(c->d_coef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice, c->stream));
    // chunks of the per-case sums of the cases of more than PERRK_RED_CHUNK elements
    std::vector<int64_t> chunk_range;
    std::vector<int32_t> case_chunk(c->n_cases + 1, 0);
    for (int cs = 0; cs < c->n_cases; ++cs) {
        case_chunk[cs] = (int32_t)(chunk_range.size() / 2);
        const int64_t b = c->case_off[cs], e = c->case_off[cs + 1];
        if (e - b > PERRK_RED_CHUNK)
            for (int64_t k = b; k < e; k += PERRK_RED_CHUNK) {
                chunk_range.push_back(k);
                chunk_range.push_back(std::min<int64_t>(e, k + PERRK_RED_CHUNK));
            }
    }
    case_chunk[c->n_cases] = (int32_t)(chunk_range.size() / 2);
    if (!chunk_range.empty()) {
        const size_t nch = chunk_range.size() / 2;
        HIPINIT(hipMalloc(&c->d_chunk_range, sizeof(int64_t) * chunk_range.size()));
        HIPINIT(hipMalloc(&c->d_case_chunk, sizeof(int32_t) * case_chunk.size()));
        HIPINIT(hipMalloc(&c->d_chunk_sums, sizeof(double) * (PERRK_MAXB + 4) * nch));
        HIPINIT(hipMemcpyAsync(c->d_chunk_range, chunk_range.data(), sizeof(int64_t) * chunk_range.size(),
                               hipMemcpyHostToDevice, c->stream));
        HIPINIT(hipMemcpyAsync(c->d_case_chunk, case_chunk.data(), sizeof(int32_t) * case_chunk.size(),
                               hipMemcpyHostToDevice, c->stream));
        c->chunks.n_chunks = (int)nch;
        c->chunks.range = c->d_chunk_range;
        c->chunks.case_chunk = c->d_case_chunk;
        c->chunks.sums = c->d_chunk_sums;
        HIPINIT(hipStreamSynchronize(c->stream));  // (the host vectors end here)
    }
    HIPINIT(launch_init_cases(c->d_cs, c->n_cases, c->stream));
    HIPINIT(launch_clear_err(c->d_err, ERR_WORDS, c->stream));
    HIPINIT(hipStreamSynchronize(c->stream));
#undef HIPINIT
    *out = c;
    return PERRK_OK;
}

int perrk_step(perrk_ctx *c, void *u_dev, const double *dt, perrk_step_info *info)
{
    if (!c || !u_dev || !dt) return fail(c, PERRK_EINVAL, "null argument");
    for (int i = 0; i < c->n_cases; ++i)
        if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return fail(c, PERRK_EINVAL, "dt[%d] must be > 0", i);
    // order after the caller's work
    HIPCHECK(c, hipEventRecord(c->ev_in, c->user_stream));
    HIPCHECK(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
    // dt upload through a ring of pinned buffers
    const int slot = c->ring;
    c->ring = (c->ring + 1) % perrk_ctx::NRING;
    HIPCHECK(c, hipEventSynchronize(c->ring_ev[slot]));
    double *hdt = c->h_dt + (size_t)slot * c->n_cases;
    double *ddt = c->d_dt + (size_t)slot * c->n_cases;
    std::memcpy(hdt, dt, sizeof(double) * c->n_cases);
    HIPCHECK(c, hipMemcpyAsync(ddt, hdt, sizeof(double) * c->n_cases, hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipEventRecord(c->ring_ev[slot], c->stream));
    HIPCHECK(c, launch_set_dt(c->d_cs, ddt, c->n_cases, c->stream));
    if (c->opt.tune == 1 && !c->tuned) {
        const int st = autotune(c, static_cast<double *>(u_dev));
        if (st != PERRK_OK) return st;
    }
    if (c->opt.use_graph && !c->profiling) {
        if (!c->gexec || c->graph_u != u_dev) {
            if (c->gexec) {
                (void)hipGraphExecDestroy(c->gexec);
                c->gexec = nullptr;
            }
            if (c->graph) {
                (void)hipGraphDestroy(c->graph);
                c->graph = nullptr;
            }
            HIPCHECK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            const int st = enqueue_step(c, static_cast<double *>(u_dev));
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(c->stream, &g);
            if (st != PERRK_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (ec != hipSuccess) return fail(c, PERRK_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
            c->graph = g;
            HIPCHECK(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
            c->graph_u = u_dev;
        }
        HIPCHECK(c, hipGraphLaunch(c->gexec, c->stream));
    } else {
        c->npev = 0;
        const int st = enqueue_step(c, static_cast<double *>(u_dev));
        if (st != PERRK_OK) return st;
        if (c->profiling) {
            HIPCHECK(c, hipStreamSynchronize(c->stream));
            // a residual pass moves bytes only for the cases still being solved
            HIPCHECK(c, hipMemcpy(c->h_cs, c->d_cs, sizeof(CaseState) * c->n_cases, hipMemcpyDeviceToHost));
            int pass = c->fused_first ? 1 : 0;  // evaluations before the first launched pass
            for (int k = 0; k < c->npev / 2; ++k) {
                float ms = 0.0f;
                HIPCHECK(c, hipEventElapsedTime(&ms, c->pev[2 * k], c->pev[2 * k + 1]));
                double bytes = c->pbytes[k];
                if (c->pcls[k] == PERRK_K_RESIDUAL) {
                    bytes = 0.0;
                    for (int cs = 0; cs < c->n_cases; ++cs)
                        if (c->h_cs[cs].passes > pass)
                            bytes += 16.0 * c->V * c->npe * (double)(c->case_off[cs + 1] - c->case_off[cs]);
                    ++pass;
                }
                perrk_kernel_stat &s = c->stats[c->pcls[k]];
                s.ms += ms;
                s.bytes += bytes;
                s.launches += 1;
                if (c->pstage[k] >= 0) {
                    perrk_kernel_stat &q = c->sstats[c->pstage[k]];
                    q.ms += ms;
                    q.bytes += bytes;
                    q.launches += 1;
                }
            }
            c->npev = 0;
        }
    }
    HIPCHECK(c, hipEventRecord(c->ev_out, c->stream));
    HIPCHECK(c, hipStreamWaitEvent(c->user_stream, c->ev_out, 0));
    if (!info) return PERRK_OK;
    HIPCHECK(c, hipMemcpyAsync(c->h_cs, c->d_cs, sizeof(CaseState) * c->n_cases, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipMemcpyAsync(c->h_err, c->d_err, sizeof(int32_t) * ERR_WORDS, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    int status = PERRK_OK;
    for (int i = 0; i < c->n_cases; ++i) {
        const CaseState &C = c->h_cs[i];
        perrk_step_info &I = info[i];
        I.gamma = C.gamma_acc;
        I.r = C.r;
        I.dH = C.dH;
        I.H_delta = C.H_delta;
        for (int j = 0; j < PERRK_MAXB; ++j) I.e[j] = C.e[j];
        I.t = C.t;
        I.passes = C.passes;
        I.flags = C.flags;
        if (C.flags & PERRK_FLAG_FALLBACK) status = PERRK_WARN_FALLBACK;
    }
    // err[ERR_PENDING] holds this step's error and those of earlier steps that
    // did not synchronise; reporting clears it
    const int e_now = c->h_err[ERR_STEP], e_all = c->h_err[ERR_PENDING];
    if (e_all) {
        HIPCHECK(c, launch_clear_err(c->d_err + ERR_PENDING, 1, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        const int e = e_now ? e_now : e_all;
        const char *what = (e & 1) ? "non-physical state (rho <= 0 or p <= 0)" : "non-finite state";
        const int code = (e & 1) ? PERRK_ENONPHYS : PERRK_ENONFINITE;
        if (e_now) return fail(c, code, "%s formed; u unmodified, step rejected", what);
        return fail(c, code, "%s formed in an earlier step called without info (that step was rejected and "
                    "left u unmodified); this step completed", what);
    }
    return status;
}

int perrk_entropy(perrk_ctx *c, const void *u_dev, double *H)
{
    if (!c || !u_dev || !H) return fail(c, PERRK_EINVAL, "null argument");
    HIPCHECK(c, hipEventRecord(c->ev_in, c->user_stream));
    HIPCHECK(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
    HIPCHECK(c, launch_clear_err(c->d_err + ERR_ENTROPY, 1, c->stream));
    HIPCHECK(c, launch_entropy(c->dim, c->sys, static_cast<const double *>(u_dev), c->d_elem, c->d_partial, c->d_H,
                               c->d_case_off, c->n_cases, c->nelem, c->gam, c->d_err + ERR_ENTROPY, c->stream));
    HIPCHECK(c, hipMemcpyAsync(c->h_H, c->d_H, sizeof(double) * c->n_cases, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipMemcpyAsync(c->h_err + ERR_ENTROPY, c->d_err + ERR_ENTROPY, sizeof(int32_t),
                               hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    std::memcpy(H, c->h_H, sizeof(double) * c->n_cases);
    const int e = c->h_err[ERR_ENTROPY];
    if (e & 1) return fail(c, PERRK_ENONPHYS, "entropy of a non-physical state (rho <= 0 or p <= 0)");
    if (e) return fail(c, PERRK_ENONFINITE, "entropy of a non-finite state");
    return PERRK_OK;
}

int perrk_rhs(perrk_ctx *c, const void *u_dev, void *k_dev)
{
    if (!c || !u_dev || !k_dev) return fail(c, PERRK_EINVAL, "null argument");
    HIPCHECK(c, hipEventRecord(c->ev_in, c->user_stream));
    HIPCHECK(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
    StageArgs a{};
    a.U = static_cast<const double *>(u_dev);
    a.K1 = k_dev;
    a.Kp = k_dev;
    a.Kout = k_dev;
    a.elem = c->d_elem;
    a.active = c->d_active;
    a.n_active = (int32_t)c->nelem;
    a.cs = c->d_cs;
    a.err = c->d_err + ERR_RHS;  // never read: the right-hand side reports no error
    a.nelem = c->nelem;
    a.gam = c->gam;
    a.gm1 = c->gam - 1.0;
    a.inv_gm1 = 1.0 / (c->gam - 1.0);
    a.flux = c->flux;
    a.volume = c->volume;
    a.sys = c->sys;
    a.c_h = c->c_h;
    a.viscous = c->viscous;
    a.mu = c->mu;
    a.prandtl = c->prandtl;
    a.grad = c->d_grad;
    a.active_all = c->d_active;
    a.n_all = (int32_t)c->nelem;
    a.c_stage = 0.0;
    a.x_lo = c->x_lo;
    a.x_hi = c->x_hi;
    HIPCHECK(c, launch_stage(c->dim, c->precision == PERRK_FP64 ? 0 : 1, c->flux, SK_FIRST, a, c->d_coef,
                             c->cfg, c->stream));
    HIPCHECK(c, hipEventRecord(c->ev_out, c->stream));
    HIPCHECK(c, hipStreamWaitEvent(c->user_stream, c->ev_out, 0));
    return PERRK_OK;
}

int perrk_get_relaxation_state(perrk_ctx *c, double *gamma_prev, double *h_offset, double *t,
                               double *gamma_hist, int32_t *n_steps)
{
    if (!c) return PERRK_EINVAL;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipMemcpy(c->h_cs, c->d_cs, sizeof(CaseState) * c->n_cases, hipMemcpyDeviceToHost));
    for (int i = 0; i < c->n_cases; ++i) {
        const CaseState &C = c->h_cs[i];
        if (gamma_prev) gamma_prev[i] = C.gamma_prev;
        if (h_offset) h_offset[i] = C.offset;
        if (t) t[i] = C.t;
        if (gamma_hist)
            for (int j = 0; j < 3; ++j) gamma_hist[3 * i + j] = C.ghist[j];
        if (n_steps) n_steps[i] = C.nsteps;
    }
    return PERRK_OK;
}

int perrk_set_relaxation_state(perrk_ctx *c, const double *gamma_prev, const double *h_offset, const double *t,
                               const double *gamma_hist, const int32_t *n_steps)
{
    if (!c) return PERRK_EINVAL;
    for (int i = 0; i < c->n_cases; ++i) {  // validate everything before changing anything
        if (gamma_prev && !(gamma_prev[i] > 0.0 && std::isfinite(gamma_prev[i])))
            return fail(c, PERRK_EINVAL, "gamma_prev[%d] must be finite and > 0", i);
        if (n_steps && n_steps[i] < 0) return fail(c, PERRK_EINVAL, "n_steps[%d] must be >= 0", i);
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipMemcpy(c->h_cs, c->d_cs, sizeof(CaseState) * c->n_cases, hipMemcpyDeviceToHost));
    for (int i = 0; i < c->n_cases; ++i) {
        CaseState &C = c->h_cs[i];
        if (gamma_prev) C.gamma_prev = gamma_prev[i];
        if (h_offset) C.offset = h_offset[i];
        if (t) C.t = t[i];
        if (gamma_hist)
            for (int j = 0; j < 3; ++j) C.ghist[j] = gamma_hist[3 * i + j];
        if (n_steps) C.nsteps = n_steps[i];
    }
    HIPCHECK(c, hipMemcpy(c->d_cs, c->h_cs, sizeof(CaseState) * c->n_cases, hipMemcpyHostToDevice));
    return PERRK_OK;
}

int perrk_set_guess_model(perrk_ctx *c, const float *weights, const float *mean, const float *scale)
{
    if (!c || !weights || !mean || !scale) return fail(c, PERRK_EINVAL, "null argument");
    std::vector<float> buf(PERRK_MLP_NW + 18, 0.0f);
    std::memcpy(buf.data(), weights, sizeof(float) * (PERRK_MLP_NW + 2));
    std::memcpy(buf.data() + PERRK_MLP_NW, mean, sizeof(float) * 8);
    std::memcpy(buf.data() + PERRK_MLP_NW + 8, scale, sizeof(float) * 8);
    // output scale and shift follow the 1377 network weights in `weights`
    // (weights[1377], weights[1378])
    buf[PERRK_MLP_NW + 16] = weights[PERRK_MLP_NW];
    buf[PERRK_MLP_NW + 17] = weights[PERRK_MLP_NW + 1];
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipMemcpy(c->d_mlp, buf.data(), sizeof(float) * buf.size(), hipMemcpyHostToDevice));
    c->have_mlp = true;
    if (c->gexec) {  // the captured graph holds the old model pointer state; recapture
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    return PERRK_OK;
}

int perrk_set_profiling(perrk_ctx *c, int on)
{
    if (!c) return PERRK_EINVAL;
    if (on && !c->pev[0])
        for (auto &e : c->pev) HIPCHECK(c, hipEventCreate(&e));
    c->profiling = on != 0;
    return PERRK_OK;
}

int perrk_get_kernel_stats(perrk_ctx *c, perrk_kernel_stat *stats, int reset)
{
    if (!c || !stats) return PERRK_EINVAL;
    std::memcpy(stats, c->stats, sizeof c->stats);
    if (reset) std::memset(c->stats, 0, sizeof c->stats);
    return PERRK_OK;
}

int perrk_get_stage_stats(perrk_ctx *c, perrk_kernel_stat *stats, int n_stages, int reset)
{
    if (!c || !stats || n_stages != c->S) return PERRK_EINVAL;
    std::memcpy(stats, c->sstats.data(), sizeof(perrk_kernel_stat) * c->S);
    if (reset) c->sstats.assign(c->S, perrk_kernel_stat{});
    return PERRK_OK;
}

int perrk_get_tuning(perrk_ctx *c, char *buf, size_t len)
{
    static const char *const flux_names[] = {"ec", "hll", "llf", "hlle", "hllc", "central"};
    if (!c || !buf || !len) return PERRK_EINVAL;
    std::string w, od;
    for (const LaunchCfg &x : c->scfg) {
        w += (w.empty() ? "" : ",") + std::to_string(x.epb_mult);
        od += (od.empty() ? "" : ",") + std::to_string(x.one_dir);
    }
    std::snprintf(buf, len,
                  "system=%s dim=%d precision=%s flux=%s volume=%s tile=%s stage_waves_per_workgroup=[%s] "
                  "stage_one_direction_at_a_time=[%s] fast_passes=%d graph=%d %s",
                  c->sys == PERRK_SYSTEM_GLM_MHD ? "glm_mhd" : "euler", c->dim,
                  c->precision == PERRK_MIXED ? "mixed" : (c->precision == PERRK_MIXED_ALL ? "mixed_all" : "fp64"),
                  flux_names[c->flux], c->volume ? "weak" : "flux_differencing", tile_name(c->dim, c->tile), w.c_str(),
                  od.c_str(), c->opt.fast_passes, c->opt.use_graph, c->tuned ? c->tune_report.c_str() : "(not tuned)");
    return PERRK_OK;
}

const char *perrk_last_error(const perrk_ctx *c) { return c ? c->err.c_str() : ""; }

const char *perrk_version(void) { return "perrk 0.1 (gfx950)"; }

void perrk_destroy(perrk_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

}  // extern "C"
