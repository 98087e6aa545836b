// Host side of the C ABI: plan construction (MLP coefficient table in FP64),
// argument validation and dispatch to the HIP launchers.  Every check runs
// before anything is enqueued on the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "pct_internal.h"
#include "pct_sort.h"

namespace pct {

static thread_local int g_last_hip_error = 0;

static int hip_status(int err)
{
    if (err == 0) return PCT_OK;
    g_last_hip_error = err;
    return PCT_ERR_HIP;
}

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

Layout layout_for(int64_t nvox, int K, int dtype)
{
    // Offsets do not depend on the value type: the accumulator always has room
    // for FP64 values, so one workspace serves both value types.
    (void)dtype;
    Layout L{};
    const size_t vsize = 8;
    size_t off = 0;
    L.hdr = off;
    off += 256;
    L.table = off;
    off = align256(off + size_t(K + 1) * kRowDoubles * sizeof(double));
    L.acc = off;
    L.acc_stride = align256(size_t(nvox + 4) * vsize);  // +4: the commit reads words in groups of 4
    off = align256(off + 3 * L.acc_stride);
    L.cnt = off;
    off = align256(off + size_t(nvox) * sizeof(int32_t));
    L.x1 = off;
    off = align256(off + size_t(nvox) * sizeof(double));
    L.partial = off;
    off = align256(off + size_t(kMaxPartials) * sizeof(double));
    L.lo = off;
    off = align256(off + size_t(nvox) * sizeof(float));
    L.total = off;
    return L;
}

GridDev grid_dev(const pct_grid &g)
{
    GridDev d{};
    const int32_t n[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        d.n[a] = n[a];
        d.pitch[a] = g.pitch[a];
        d.inv_pitch[a] = 1.0 / g.pitch[a];
        d.inv_n[a] = 1.0 / double(n[a]);
        d.lo[a] = g.origin[a];
        d.hi[a] = g.origin[a] + n[a] * g.pitch[a];
    }
    d.inv_nxy = 1.0 / (double(n[0]) * double(n[1]));
    return d;
}

PathSrc path_src(const pct_plan &pl, const void *table_dev)
{
    PathSrc p{};
    p.tab = static_cast<const double *>(table_dev);
    p.K = pl.K;
    p.nvmax = path_vertices_max(pl);
    p.hull = pl.hull;
    p.hx = pl.hull_c[0];
    p.hy = pl.hull_c[1];
    p.hr = pl.hull_r;
    p.u_in = pl.mlp.u_in;
    p.u_out = pl.mlp.u_out;
    p.step = pl.mlp.step;
    for (int k = 0; k < 6; ++k) p.poly[k] = pl.mlp.poly[k];
    p.E0 = pl.mlp.E0;
    p.X0 = pl.mlp.X0;
    p.log_term = pl.mlp.log_term;
    return p;
}

// tracker segment, hull-to-hull MLP (at most K segments), tracker segment
int path_vertices_max(const pct_plan &pl) { return pl.K + 1 + (pl.hull ? 2 : 0); }

// ---------------------------------------------------------------------------
// MLP coefficient table
//
// Scattering matrix of the path from depth lo to depth `end` (cm), seen at
// `end`:  S = E0^2 l(end - lo) / X0 * [[J2, J1], [J1, J0]],
//         J_m = integral over [lo, end] of (end - s)^m P(s) ds,
// P the 1/(beta^2 p^2) polynomial and l(L) = (1 + 0.038 ln(L/X0))^2 (optional).
// J_m is evaluated with 4-point Gauss-Legendre quadrature, exact for the
// degree <= 7 integrand.
//
// The most likely position at depth d given the entry state y0 = (t, th) and
// the exit state y2 is the Gaussian posterior mean with prior R0 y0, prior
// covariance S1 = S(0 -> d) and observation y2 = R1 y1 + N(0, S2),
// S2 = S(d -> D):  y1 = (I - G R1) R0 y0 + G y2,  G = S1 R1^T (R1 S1 R1^T + S2)^-1.
// This is algebraically the same as (S1^-1 + R1^T S2^-1 R1)^-1 (S1^-1 R0 y0 +
// R1^T S2^-1 y2) (Schulte et al. 2008) but needs no inverse of the nearly
// singular S1 close to the entry plane.
// ---------------------------------------------------------------------------
static double poly_at(const pct_mlp &m, double s)
{
    double v = 0.0;
    for (int k = 5; k >= 0; --k) v = v * s + m.poly[k];
    return v;
}

static void scatter_matrix(const pct_mlp &m, double lo, double end, double S[4])
{
    static const double r1 = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    static const double r2 = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    static const double w1 = (18.0 + std::sqrt(30.0)) / 36.0;
    static const double w2 = (18.0 - std::sqrt(30.0)) / 36.0;
    const double xs[4] = {-r2, -r1, r1, r2};
    const double ws[4] = {w2, w1, w1, w2};
    double h = 0.5 * (end - lo), c = 0.5 * (end + lo);
    double J0 = 0, J1 = 0, J2 = 0;
    for (int i = 0; i < 4; ++i) {
        double s = c + h * xs[i];
        double w = ws[i] * h * poly_at(m, s);
        double e = end - s;
        J0 += w;
        J1 += w * e;
        J2 += w * e * e;
    }
    double f = m.E0 * m.E0 / m.X0;
    if (m.log_term) {
        double l = 1.0 + 0.038 * std::log((end - lo) / m.X0);
        f *= l * l;
    }
    S[0] = f * J2;
    S[1] = f * J1;
    S[2] = f * J1;
    S[3] = f * J0;
}

static bool build_table(pct_plan &pl)
{
    const pct_mlp &m = pl.mlp;
    const double D = m.u_out - m.u_in;
    const int K = pl.K;
    pl.table.assign(size_t(K + 1) * kRowDoubles, 0.0);
    const double Dcm = D / 10.0;
    for (int k = 0; k <= K; ++k) {
        double *r = &pl.table[size_t(k) * kRowDoubles];
        double dk = k * m.step;
        if (!(dk < D)) dk = D;
        r[4] = m.u_in + dk;
        if (k == 0) { r[0] = 1.0; continue; }
        if (k == K) { r[2] = 1.0; continue; }
        double d = dk / 10.0;
        double S1[4], S2[4];
        scatter_matrix(m, 0.0, d, S1);
        scatter_matrix(m, d, Dcm, S2);
        // both scattering matrices must be covariances (positive definite)
        for (const double *S : {S1, S2})
            if (!(S[0] > 0.0) || !(S[3] > 0.0) || !(S[0] * S[3] - S[1] * S[2] > 0.0)) return false;
        const double e = Dcm - d;  // R1 = [[1, e], [0, 1]], R0 = [[1, d], [0, 1]]
        // T = R1 S1 R1^T + S2
        double a = S1[0] + 2.0 * e * S1[1] + e * e * S1[3] + S2[0];
        double b = S1[1] + e * S1[3] + S2[1];
        double dd = S1[3] + S2[3];
        double det = a * dd - b * b;
        double Ti[4] = {dd / det, -b / det, -b / det, a / det};
        // S1 R1^T = [[S1_00 + e S1_01, S1_01], [S1_10 + e S1_11, S1_11]]
        double U[4] = {S1[0] + e * S1[1], S1[1], S1[2] + e * S1[3], S1[3]};
        double G[4] = {U[0] * Ti[0] + U[1] * Ti[2], U[0] * Ti[1] + U[1] * Ti[3],
                       U[2] * Ti[0] + U[3] * Ti[2], U[2] * Ti[1] + U[3] * Ti[3]};
        // (I - G R1) R0, first row: [1 - G00, -(G00 e) - G01 + 0] * R0
        double q0 = 1.0 - G[0];
        double q1 = -G[0] * e - G[1];
        double c0t = q0;
        double c0th = q0 * d + q1;
        r[0] = c0t;
        r[1] = c0th * 10.0;
        r[2] = G[0];
        r[3] = G[1] * 10.0;
    }
    for (double v : pl.table)
        if (!std::isfinite(v)) return false;
    return true;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

static int check_grid_mlp(const pct_grid *g, const pct_mlp *m)
{
    if (!g || !m) return PCT_ERR_INVALID_ARG;
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return PCT_ERR_INVALID_ARG;
    if (int64_t(g->nx) * g->ny * g->nz >= (int64_t(1) << 31)) return PCT_ERR_INVALID_ARG;
    for (int a = 0; a < 3; ++a)
        if (!finite_pos(g->pitch[a]) || !std::isfinite(g->origin[a])) return PCT_ERR_INVALID_ARG;
    if (!std::isfinite(m->u_in) || !std::isfinite(m->u_out) || !(m->u_in < m->u_out)) return PCT_ERR_INVALID_ARG;
    if (!finite_pos(m->step) || !finite_pos(m->E0) || !finite_pos(m->X0)) return PCT_ERR_INVALID_ARG;
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(m->poly[k])) return PCT_ERR_INVALID_ARG;
    if (m->log_term != 0 && m->log_term != 1) return PCT_ERR_INVALID_ARG;
    double K = std::ceil((m->u_out - m->u_in) / m->step);
    if (!(K >= 1.0) || K > kMaxSegments) return PCT_ERR_INVALID_ARG;
    return PCT_OK;
}

static int check_protons(const pct_protons *p)
{
    if (!p || p->n < 0) return PCT_ERR_INVALID_ARG;
    if (p->n > (int64_t(1) << 40)) return PCT_ERR_INVALID_ARG;
    if (p->n == 0) return PCT_OK;
    const float *ptrs[9] = {p->t_in, p->v_in, p->th_in, p->ph_in, p->t_out, p->v_out, p->th_out, p->ph_out,
                            p->gantry};
    for (const float *q : ptrs)
        if (!q) return PCT_ERR_INVALID_ARG;
    return PCT_OK;
}

static ProtonsDev protons_dev(const pct_protons *p)
{
    return ProtonsDev{p->t_in, p->v_in, p->th_in, p->ph_in, p->t_out, p->v_out, p->th_out, p->ph_out, p->gantry};
}

static int check_ws(const pct_plan *pl, void *ws, size_t ws_bytes, int dtype)
{
    if (!ws) return PCT_ERR_WORKSPACE;
    Layout L = layout_for(pl->nvox, pl->K, dtype);
    if (ws_bytes < L.total) return PCT_ERR_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return PCT_ERR_WORKSPACE;
    for (int i = 0; i < pl->n_uploaded; ++i)
        if (pl->uploaded[i] == ws) return PCT_OK;
    return PCT_ERR_WORKSPACE;
}

static bool valid_dtype(int32_t d) { return d == PCT_F32 || d == PCT_F64; }

FbpLayout fbp_layout(int64_t nbins)
{
    FbpLayout L{};
    size_t off = 0;
    L.sum = off;
    off = align256(off + size_t(nbins) * sizeof(uint64_t));
    L.cnt = off;
    off = align256(off + size_t(nbins) * sizeof(uint32_t));
    L.proj = off;
    off = align256(off + size_t(nbins) * sizeof(double));
    L.q = off;
    off = align256(off + size_t(nbins) * sizeof(double));
    L.total = off;
    return L;
}

// Validated FBP geometry of a plan; nbins receives nz * n_angles * n_t.
static int fbp_geometry(const pct_plan *plan, const pct_fbp_geom *geom, FbpDev &f, int64_t &nbins)
{
    if (!plan || !geom) return PCT_ERR_INVALID_ARG;
    if (geom->n_angles < 1 || geom->n_angles > kFbpMaxAngles) return PCT_ERR_INVALID_ARG;
    if (geom->n_t < 1 || geom->n_t > kFbpMaxLateral) return PCT_ERR_INVALID_ARG;
    if (!std::isfinite(geom->t0) || !finite_pos(geom->dt)) return PCT_ERR_INVALID_ARG;
    nbins = int64_t(plan->grid.nz) * geom->n_angles * geom->n_t;
    if (nbins >= (int64_t(1) << 31)) return PCT_ERR_INVALID_ARG;
    f = FbpDev{};
    f.n_ang = geom->n_angles;
    f.n_t = geom->n_t;
    f.nz = plan->grid.nz;
    f.t0 = geom->t0;
    f.dt = geom->dt;
    f.dphi = 2.0 * M_PI / geom->n_angles;
    f.w = -plan->mlp.u_in / (plan->mlp.u_out - plan->mlp.u_in);
    f.z0 = plan->grid.origin[2];
    f.pz = plan->grid.pitch[2];
    return PCT_OK;
}

static bool disjoint(const void *a, size_t na, const void *b, size_t nb)
{
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa + na <= pb || pb + nb <= pa;
}

}  // namespace pct

using namespace pct;

extern "C" {

int pct_plan_create(const pct_grid *grid, const pct_mlp *mlp, pct_plan **out)
{
    if (!out) return PCT_ERR_INVALID_ARG;
    *out = nullptr;
    int st = check_grid_mlp(grid, mlp);
    if (st) return st;
    pct_plan *pl = new (std::nothrow) pct_plan();
    if (!pl) return PCT_ERR_INVALID_ARG;
    pl->grid = *grid;
    pl->mlp = *mlp;
    pl->K = int(std::ceil((mlp->u_out - mlp->u_in) / mlp->step));
    if (pl->K < 1) pl->K = 1;
    pl->nvox = int64_t(grid->nx) * grid->ny * grid->nz;
    pl->n_uploaded = 0;
    pl->prof_used[0] = pl->prof_used[1] = 0;
    pl->graph_exec = nullptr;
    pl->capture_stream = nullptr;
    pl->cancel_stream = nullptr;
    if (!build_table(*pl)) {
        delete pl;
        return PCT_ERR_INVALID_ARG;
    }
    *out = pl;
    return PCT_OK;
}

void pct_plan_destroy(pct_plan *plan)
{
    if (!plan) return;
    profile_release(*plan);
    graph_release(*plan);
    delete plan;
}

int pct_plan_set_hull(pct_plan *plan, const pct_hull *hull)
{
    if (!plan) return PCT_ERR_INVALID_ARG;
    if (hull && !(finite_pos(hull->radius) && std::isfinite(hull->cx) && std::isfinite(hull->cy)))
        return PCT_ERR_INVALID_ARG;
    graph_release(*plan);  // recorded sweeps use the other kernels
    plan->hull = hull ? 1 : 0;
    plan->hull_c[0] = hull ? hull->cx : 0.0;
    plan->hull_c[1] = hull ? hull->cy : 0.0;
    plan->hull_r = hull ? hull->radius : 0.0;
    return PCT_OK;
}

int pct_plan_segments(const pct_plan *plan, int32_t *K)
{
    if (!plan || !K) return PCT_ERR_INVALID_ARG;
    *K = plan->K;
    return PCT_OK;
}

int pct_plan_table(const pct_plan *plan, double *tab, int64_t tab_len)
{
    if (!plan || !tab || tab_len < int64_t(plan->K + 1) * 4) return PCT_ERR_INVALID_ARG;
    for (int k = 0; k <= plan->K; ++k)
        for (int c = 0; c < 4; ++c) tab[k * 4 + c] = plan->table[size_t(k) * kRowDoubles + c];
    return PCT_OK;
}

int pct_workspace_size(const pct_plan *plan, int64_t n, int32_t dtype, size_t *bytes)
{
    if (!plan || !bytes || n < 0 || !valid_dtype(dtype)) return PCT_ERR_INVALID_ARG;
    const int nslab = std::max(plan->grid.nx, plan->grid.ny);
    *bytes = layout_for(plan->nvox, plan->K, dtype).total + (n > 0 ? 2 * slot_bytes(n) + bin_bytes(n, nslab) : 0);
    return PCT_OK;
}

int pct_plan_upload(pct_plan *plan, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan) return PCT_ERR_INVALID_ARG;
    if (!ws) return PCT_ERR_WORKSPACE;
    if (ws_bytes < layout_for(plan->nvox, plan->K, PCT_F32).total) return PCT_ERR_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return PCT_ERR_WORKSPACE;
    int st = hip_status(upload_table(*plan, ws, stream));
    if (st) return st;
    bool known = false;
    for (int i = 0; i < plan->n_uploaded; ++i) known |= plan->uploaded[i] == ws;
    if (!known) {
        if (plan->n_uploaded == kMaxUploads) {
            for (int i = 1; i < kMaxUploads; ++i) plan->uploaded[i - 1] = plan->uploaded[i];
            plan->n_uploaded--;
        }
        plan->uploaded[plan->n_uploaded++] = ws;
    }
    return PCT_OK;
}

int pct_device_status(const pct_plan *plan, void *ws, size_t ws_bytes, int reset, uint32_t *bits, void *stream)
{
    if (!plan || !bits) return PCT_ERR_INVALID_ARG;
    int st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    return hip_status(read_status(*plan, ws, reset, bits, stream));
}

int pct_mlp_trace(const pct_plan *plan, const pct_protons *p, int64_t first, int64_t count, int32_t max_nnz,
                  int32_t *vox, double *chord, int32_t *nnz, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan) return PCT_ERR_INVALID_ARG;
    int st = check_protons(p);
    if (st) return st;
    if (first < 0 || count < 0 || first + count > p->n || max_nnz <= 0) return PCT_ERR_INVALID_ARG;
    if (count > 0 && (!vox || !chord || !nnz)) return PCT_ERR_INVALID_ARG;
    if (count * int64_t(max_nnz) >= (int64_t(1) << 40)) return PCT_ERR_INVALID_ARG;
    st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    if (count == 0) return PCT_OK;
    return hip_status(launch_trace(*plan, protons_dev(p), first, count, max_nnz, vox, chord, nnz, ws, stream));
}

int pct_forward(const pct_plan *plan, const pct_protons *p, const void *x, int32_t dtype, void *y, void *nrm2,
                void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !valid_dtype(dtype)) return PCT_ERR_INVALID_ARG;
    int st = check_protons(p);
    if (st) return st;
    if (p->n > 0 && (!x || !y)) return PCT_ERR_INVALID_ARG;
    st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    if (p->n == 0) return PCT_OK;
    return hip_status(launch_forward(*plan, protons_dev(p), p->n, x, dtype, y, nrm2, ws, stream));
}

int pct_backproject(const pct_plan *plan, const pct_protons *p, const void *r, int32_t dtype, void *g, void *ws,
                    size_t ws_bytes, void *stream)
{
    if (!plan || !valid_dtype(dtype)) return PCT_ERR_INVALID_ARG;
    int st = check_protons(p);
    if (st) return st;
    if (p->n > 0 && (!r || !g)) return PCT_ERR_INVALID_ARG;
    st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    if (p->n == 0) return PCT_OK;
    return hip_status(launch_backproject(*plan, protons_dev(p), p->n, r, dtype, g, ws, stream));
}

int pct_drop_iterate(const pct_plan *plan, const pct_protons *p, const float *b, void *x,
                     const pct_drop_opts *o, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !o) return PCT_ERR_INVALID_ARG;
    int st = check_protons(p);
    if (st) return st;
    if (!x) return PCT_ERR_INVALID_ARG;
    if (p->n > 0 && !b) return PCT_ERR_INVALID_ARG;
    if (o->block <= 0 || !finite_pos(o->lambda) || o->n_iter < 0 || !valid_dtype(o->dtype)) return PCT_ERR_INVALID_ARG;
    if (o->chord < PCT_CHORD_F64 || o->chord > PCT_CHORD_BF16) return PCT_ERR_INVALID_ARG;
    if (o->flags & ~(PCT_DROP_CHECK_FINITE | PCT_DROP_NO_GRAPH | PCT_DROP_PROFILE | PCT_DROP_SEPARATE_COMMIT |
                     PCT_DROP_NO_TRACE_AHEAD | PCT_DROP_FUSED_COMMIT | PCT_DROP_NO_COMPENSATION |
                     PCT_DROP_CANCELLABLE | PCT_DROP_DETERMINISTIC))
        return PCT_ERR_INVALID_ARG;
    if (o->block > (int64_t(1) << 31)) return PCT_ERR_INVALID_ARG;
    if ((o->dtype == PCT_F32 || (o->flags & PCT_DROP_DETERMINISTIC)) && o->block >= (int64_t(1) << 19))
        return PCT_ERR_INVALID_ARG;
    if (o->lanes != 0 && o->lanes != 1 && o->lanes != 8 && o->lanes != 16 && o->lanes != 32 && o->lanes != 64)
        return PCT_ERR_INVALID_ARG;
    if (o->reserved != 0) return PCT_ERR_INVALID_ARG;
    int64_t T = p->n > 0 ? (p->n + o->block - 1) / o->block : 0;
    int64_t end = o->block_end < 0 ? T : o->block_end;
    if (o->block_begin < 0 || end > T || o->block_begin > end) return PCT_ERR_INVALID_ARG;
    st = check_ws(plan, ws, ws_bytes, o->dtype);
    if (st) return st;
    if (o->n_iter == 0 || o->block_begin == end)
        return (o->flags & PCT_DROP_CANCELLABLE) ? hip_status(launch_gate_reset(*plan, ws, stream)) : PCT_OK;
    pct_drop_opts oo = *o;
    oo.block_end = end;
    // the plan's geometry is immutable; its sweep-graph cache and profiling
    // events are not, and calls sharing the plan take turns on them
    pct_plan &pl = *const_cast<pct_plan *>(plan);
    std::lock_guard<std::mutex> lock(pl.mu);
    return hip_status(launch_drop(pl, protons_dev(p), p->n, b, x, oo, ws, ws_bytes, stream));
}

int pct_drop_cancel(pct_plan *plan, void *ws, size_t ws_bytes, int32_t request)
{
    if (!plan || !ws) return PCT_ERR_INVALID_ARG;
    int st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    return hip_status(write_cancel(*plan, ws, request));
}

int pct_drop_progress(const pct_plan *plan, void *ws, size_t ws_bytes, int64_t *blocks_done, void *stream)
{
    if (!plan || !ws || !blocks_done) return PCT_ERR_INVALID_ARG;
    int st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    int halted = 0;
    st = hip_status(read_progress(*plan, ws, blocks_done, &halted, stream));
    if (st) return st;
    return halted ? PCT_ERR_CANCELLED : PCT_OK;
}

int pct_tv(const pct_plan *plan, const void *x, int32_t dtype, double eps, double *value_dev, void *grad,
           void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !x || !value_dev || !finite_pos(eps) || !valid_dtype(dtype)) return PCT_ERR_INVALID_ARG;
    int st = check_ws(plan, ws, ws_bytes, dtype);
    if (st) return st;
    return hip_status(launch_tv(*plan, x, dtype, eps, value_dev, grad, ws, stream));
}

int pct_tv_static(const pct_plan *plan, const void *x, int32_t dtype, double eps, double *value_dev, void *grad,
                  void *stream)
{
    if (!plan || !x || !value_dev || !finite_pos(eps) || !valid_dtype(dtype)) return PCT_ERR_INVALID_ARG;
    return hip_status(launch_tv_static(*plan, x, dtype, eps, value_dev, grad, stream));
}

int pct_rows_count(const pct_plan *plan, const pct_protons *p, int64_t *offsets, void *ws, size_t ws_bytes,
                   void *stream)
{
    if (!plan || !offsets) return PCT_ERR_INVALID_ARG;
    int st = check_protons(p);
    if (st) return st;
    st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    return hip_status(launch_rows_count(*plan, protons_dev(p), p->n, offsets, ws, stream));
}

static bool stored_chord_type(int32_t c) { return c == PCT_CHORD_F32 || c == PCT_CHORD_F16 || c == PCT_CHORD_BF16; }

int pct_rows_build(const pct_plan *plan, const pct_protons *p, int32_t chord_type, const int64_t *offsets,
                   int32_t *vox, void *chord, double *n2, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !stored_chord_type(chord_type)) return PCT_ERR_INVALID_ARG;
    int st = check_protons(p);
    if (st) return st;
    if (p->n > 0 && (!offsets || !vox || !chord || !n2)) return PCT_ERR_INVALID_ARG;
    st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    if (p->n == 0) return PCT_OK;
    return hip_status(launch_rows_build(*plan, protons_dev(p), p->n, chord_type, offsets, vox, chord, n2, ws, stream));
}

int pct_drop_iterate_rows(const pct_plan *plan, const pct_rows *rows, const float *b, void *x,
                          const pct_drop_opts *o, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !rows || !o || !x) return PCT_ERR_INVALID_ARG;
    if (rows->n < 0 || rows->n > (int64_t(1) << 40) || rows->reserved != 0) return PCT_ERR_INVALID_ARG;
    if (!stored_chord_type(rows->chord_type)) return PCT_ERR_INVALID_ARG;
    if (rows->n > 0 && (!rows->offsets || !rows->vox || !rows->chord || !rows->n2 || !b)) return PCT_ERR_INVALID_ARG;
    if (o->block <= 0 || !finite_pos(o->lambda) || o->n_iter < 0 || !valid_dtype(o->dtype)) return PCT_ERR_INVALID_ARG;
    if (o->chord != rows->chord_type) return PCT_ERR_INVALID_ARG;
    if (o->flags & ~(PCT_DROP_CHECK_FINITE | PCT_DROP_NO_GRAPH | PCT_DROP_PROFILE | PCT_DROP_SEPARATE_COMMIT |
                     PCT_DROP_CANCELLABLE | PCT_DROP_DETERMINISTIC))
        return PCT_ERR_INVALID_ARG;
    if (o->block >= (int64_t(1) << 19)) return PCT_ERR_INVALID_ARG;
    if (o->lanes != 0 && o->lanes != 16 && o->lanes != 32 && o->lanes != 64) return PCT_ERR_INVALID_ARG;
    if (o->reserved != 0) return PCT_ERR_INVALID_ARG;
    if (o->dtype != PCT_F32 || (o->flags & (PCT_DROP_SEPARATE_COMMIT | PCT_DROP_CANCELLABLE)))
        return PCT_ERR_UNSUPPORTED;
    int64_t T = rows->n > 0 ? (rows->n + o->block - 1) / o->block : 0;
    int64_t end = o->block_end < 0 ? T : o->block_end;
    if (o->block_begin < 0 || end > T || o->block_begin > end) return PCT_ERR_INVALID_ARG;
    int st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    if (o->n_iter == 0 || o->block_begin == end) return PCT_OK;
    pct_drop_opts oo = *o;
    oo.block_end = end;
    pct_plan &pl = *const_cast<pct_plan *>(plan);
    std::lock_guard<std::mutex> lock(pl.mu);
    return hip_status(launch_drop_rows(pl, *rows, b, static_cast<float *>(x), oo, ws,
                                       stream));
}

int pct_order_blocks(const pct_plan *plan, const pct_protons *p, const float *b, int64_t block,
                     const pct_protons_buf *out, float *b_out, void *stream)
{
    if (!plan || !out) return PCT_ERR_INVALID_ARG;
    int st = check_protons(p);
    if (st) return st;
    if (block <= 0 || block > 8192) return PCT_ERR_INVALID_ARG;
    if (p->n == 0) return PCT_OK;
    if (out->capacity < p->n) return PCT_ERR_INVALID_ARG;
    float *ptrs[9] = {out->t_in, out->v_in, out->th_in, out->ph_in, out->t_out, out->v_out, out->th_out, out->ph_out,
                      out->gantry};
    for (float *q : ptrs)
        if (!q) return PCT_ERR_INVALID_ARG;
    if (b && !b_out) return PCT_ERR_INVALID_ARG;
    if ((p->n + block - 1) / block >= (int64_t(1) << 31)) return PCT_ERR_INVALID_ARG;
    ProtonsBufDev o{out->t_in, out->v_in, out->th_in, out->ph_in, out->t_out, out->v_out, out->th_out, out->ph_out,
                    out->gantry};
    return hip_status(launch_order_blocks(*plan, protons_dev(p), p->n, b, block, o, b ? b_out : nullptr, stream));
}

static int sort_setup(const pct_plan *plan, const pct_sort_opts *o, SortDev &s)
{
    if (!plan || !o) return PCT_ERR_INVALID_ARG;
    if (o->n_angles < 1 || o->n_angles > kSortMaxAngles || o->reserved != 0) return PCT_ERR_INVALID_ARG;
    if (!(o->slab_mm > 0.0) || !std::isfinite(o->slab_mm)) return PCT_ERR_INVALID_ARG;
    const double ns = std::ceil(double(plan->grid.nz) * plan->grid.pitch[2] / o->slab_mm);
    if (!(ns >= 1.0) || ns > double(kSortMaxSlabs)) return PCT_ERR_INVALID_ARG;
    auto bit_width = [](uint32_t v) {
        int w = 0;
        while (v) {
            ++w;
            v >>= 1;
        }
        return w;
    };
    s.n_angles = o->n_angles;
    s.n_slabs = int32_t(ns);
    s.bits_s = bit_width(uint32_t(s.n_slabs - 1));
    s.passes = (32 + s.bits_s + bit_width(uint32_t(s.n_angles)) + 7) / 8;
    s.dphi = 2.0 * M_PI / double(o->n_angles);
    s.z0 = plan->grid.origin[2];
    s.slab = o->slab_mm;
    return PCT_OK;
}

int pct_sort_scan_workspace_size(int64_t n, size_t *bytes)
{
    if (!bytes || n < 0 || n > kSortMaxRecords) return PCT_ERR_INVALID_ARG;
    *bytes = sort_layout(n).total;
    return PCT_OK;
}

int pct_sort_scan(const pct_plan *plan, const pct_protons *p, const float *b, const pct_sort_opts *opts,
                  const pct_protons_buf *out, float *b_out, int64_t *perm, void *ws, size_t ws_bytes, void *stream)
{
    SortDev s;
    int st = sort_setup(plan, opts, s);
    if (st) return st;
    st = check_protons(p);
    if (st) return st;
    if (!out || p->n > kSortMaxRecords) return PCT_ERR_INVALID_ARG;
    if (p->n == 0) return PCT_OK;
    if (out->capacity < p->n) return PCT_ERR_INVALID_ARG;
    float *ptrs[9] = {out->t_in, out->v_in, out->th_in, out->ph_in, out->t_out, out->v_out, out->th_out, out->ph_out,
                      out->gantry};
    for (float *q : ptrs)
        if (!q) return PCT_ERR_INVALID_ARG;
    if (b && !b_out) return PCT_ERR_INVALID_ARG;
    const SortLayout L = sort_layout(p->n);
    if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255u)) return PCT_ERR_WORKSPACE;
    ProtonsBufDev o{out->t_in, out->v_in, out->th_in, out->ph_in, out->t_out, out->v_out, out->th_out, out->ph_out,
                    out->gantry};
    return hip_status(launch_sort_scan(s, protons_dev(p), p->n, b, o, b ? b_out : nullptr, perm, ws, stream));
}

int pct_region_layout(int32_t nz, int32_t n_regions, int32_t halo, int32_t *z_lo, int32_t *z_hi, int32_t *core_lo,
                      int32_t *core_hi)
{
    if (nz < 1 || n_regions < 1 || n_regions > nz || halo < 0) return PCT_ERR_INVALID_ARG;
    if (!z_lo || !z_hi || !core_lo || !core_hi) return PCT_ERR_INVALID_ARG;
    for (int32_t r = 0; r < n_regions; ++r) {
        const int32_t c0 = int32_t(int64_t(r) * nz / n_regions);
        const int32_t c1 = int32_t(int64_t(r + 1) * nz / n_regions) - 1;
        core_lo[r] = c0;
        core_hi[r] = c1;
        z_lo[r] = r > 0 ? std::max<int32_t>(0, c0 - halo) : 0;
        z_hi[r] = r < n_regions - 1 ? int32_t(std::min<int64_t>(nz - 1, int64_t(c1) + halo)) : nz - 1;
    }
    return PCT_OK;
}

int pct_plan_region(const pct_plan *parent, int32_t z_lo, int32_t z_hi, pct_plan **out)
{
    if (!parent || !out) return PCT_ERR_INVALID_ARG;
    *out = nullptr;
    if (z_lo < 0 || z_hi < z_lo || z_hi >= parent->grid.nz) return PCT_ERR_INVALID_ARG;
    pct_grid g = parent->grid;
    g.nz = z_hi - z_lo + 1;
    g.origin[2] = parent->grid.origin[2] + double(z_lo) * parent->grid.pitch[2];
    int st = pct_plan_create(&g, &parent->mlp, out);
    if (st) return st;
    (*out)->hull = parent->hull;
    (*out)->hull_c[0] = parent->hull_c[0];
    (*out)->hull_c[1] = parent->hull_c[1];
    (*out)->hull_r = parent->hull_r;
    return PCT_OK;
}

int pct_region_select(const pct_plan *plan, const pct_protons *p, const float *b, int32_t z_lo, int32_t z_hi,
                      const pct_protons_buf *out, float *b_out, int64_t *count, void *ws, size_t ws_bytes,
                      void *stream)
{
    if (!plan || !out || !count) return PCT_ERR_INVALID_ARG;
    int st = check_protons(p);
    if (st) return st;
    if (z_lo < 0 || z_hi < z_lo || z_hi >= plan->grid.nz) return PCT_ERR_INVALID_ARG;
    if (out->capacity < 0) return PCT_ERR_INVALID_ARG;
    if (out->capacity > 0) {
        float *ptrs[9] = {out->t_in, out->v_in, out->th_in, out->ph_in, out->t_out, out->v_out, out->th_out,
                          out->ph_out, out->gantry};
        for (float *q : ptrs)
            if (!q) return PCT_ERR_INVALID_ARG;
        if (b && !b_out) return PCT_ERR_INVALID_ARG;
    }
    st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    ProtonsBufDev o{out->t_in, out->v_in, out->th_in, out->ph_in, out->t_out, out->v_out, out->th_out, out->ph_out,
                    out->gantry};
    return hip_status(launch_region_select(*plan, protons_dev(p), p->n, b, z_lo, z_hi, o, out->capacity,
                                           b ? b_out : nullptr, count, ws, stream));
}

int pct_slice_span_histogram(const pct_plan *plan, const pct_protons *p, int64_t *hist, void *ws, size_t ws_bytes,
                             void *stream)
{
    if (!plan || !hist) return PCT_ERR_INVALID_ARG;
    int st = check_protons(p);
    if (st) return st;
    if (plan->grid.nz > 16384) return PCT_ERR_UNSUPPORTED;  // bins live in LDS
    st = check_ws(plan, ws, ws_bytes, PCT_F32);
    if (st) return st;
    if (p->n == 0) return PCT_OK;
    return hip_status(launch_span_histogram(*plan, protons_dev(p), p->n, hist, stream));
}

int pct_select_slices(const pct_plan *plan, const void *src, int32_t src_z0, void *dst, int32_t dst_z0,
                      int32_t z_first, int32_t z_count, int32_t dtype, void *stream)
{
    if (!plan || !valid_dtype(dtype) || z_count < 0) return PCT_ERR_INVALID_ARG;
    if (src_z0 < 0 || dst_z0 < 0 || z_first < src_z0 || z_first < dst_z0) return PCT_ERR_INVALID_ARG;
    if (int64_t(z_first) + z_count > plan->grid.nz) return PCT_ERR_INVALID_ARG;
    if (z_count == 0) return PCT_OK;
    if (!src || !dst) return PCT_ERR_INVALID_ARG;
    const size_t plane = size_t(plan->grid.nx) * size_t(plan->grid.ny) * (dtype == PCT_F64 ? 8 : 4);
    const char *s = static_cast<const char *>(src) + size_t(z_first - src_z0) * plane;
    char *d = static_cast<char *>(dst) + size_t(z_first - dst_z0) * plane;
    return hip_status(copy_device(d, s, size_t(z_count) * plane, stream));
}

int pct_fbp_workspace_size(const pct_plan *plan, const pct_fbp_geom *geom, size_t *bytes)
{
    FbpDev f;
    int64_t nb;
    int st = fbp_geometry(plan, geom, f, nb);
    if (st) return st;
    if (!bytes) return PCT_ERR_INVALID_ARG;
    *bytes = fbp_layout(nb).total;
    return PCT_OK;
}

int pct_fbp_sinogram(const pct_plan *plan, const pct_fbp_geom *geom, const pct_protons *p, const float *b,
                     double *proj, int32_t *count, void *fbp_ws, size_t fbp_ws_bytes, void *stream)
{
    FbpDev f;
    int64_t nb;
    int st = fbp_geometry(plan, geom, f, nb);
    if (st) return st;
    st = check_protons(p);
    if (st) return st;
    if (!proj || (p->n > 0 && !b)) return PCT_ERR_INVALID_ARG;
    const FbpLayout L = fbp_layout(nb);
    if (!fbp_ws || fbp_ws_bytes < L.proj || (reinterpret_cast<uintptr_t>(fbp_ws) & 255u)) return PCT_ERR_WORKSPACE;
    char *w = static_cast<char *>(fbp_ws);
    if (!disjoint(proj, size_t(nb) * 8, w, L.proj) || (count && !disjoint(count, size_t(nb) * 4, w, L.proj)))
        return PCT_ERR_INVALID_ARG;
    return hip_status(launch_fbp_sinogram(f, protons_dev(p), p->n, b, reinterpret_cast<unsigned long long *>(w + L.sum),
                                          reinterpret_cast<unsigned *>(w + L.cnt), proj, count, stream));
}

int pct_fbp_filter(const pct_plan *plan, const pct_fbp_geom *geom, const double *proj, double *q, void *stream)
{
    FbpDev f;
    int64_t nb;
    int st = fbp_geometry(plan, geom, f, nb);
    if (st) return st;
    if (!proj || !q || !disjoint(proj, size_t(nb) * 8, q, size_t(nb) * 8)) return PCT_ERR_INVALID_ARG;
    return hip_status(launch_fbp_filter(f, proj, q, stream));
}

int pct_fbp_backproject(const pct_plan *plan, const pct_fbp_geom *geom, const double *q, void *x, int32_t dtype,
                        void *stream)
{
    FbpDev f;
    int64_t nb;
    int st = fbp_geometry(plan, geom, f, nb);
    if (st) return st;
    if (!q || !x || !valid_dtype(dtype)) return PCT_ERR_INVALID_ARG;
    const size_t xb = size_t(plan->nvox) * (dtype == PCT_F64 ? 8 : 4);
    if (!disjoint(q, size_t(nb) * 8, x, xb)) return PCT_ERR_INVALID_ARG;
    return hip_status(launch_fbp_backproject(f, grid_dev(plan->grid), q, x, dtype, stream));
}

int pct_fbp(const pct_plan *plan, const pct_fbp_geom *geom, const pct_protons *p, const float *b, void *x,
            int32_t dtype, void *fbp_ws, size_t fbp_ws_bytes, void *stream)
{
    FbpDev f;
    int64_t nb;
    int st = fbp_geometry(plan, geom, f, nb);
    if (st) return st;
    st = check_protons(p);
    if (st) return st;
    if (!x || !valid_dtype(dtype) || (p->n > 0 && !b)) return PCT_ERR_INVALID_ARG;
    const FbpLayout L = fbp_layout(nb);
    if (!fbp_ws || fbp_ws_bytes < L.total || (reinterpret_cast<uintptr_t>(fbp_ws) & 255u)) return PCT_ERR_WORKSPACE;
    char *w = static_cast<char *>(fbp_ws);
    const size_t xb = size_t(plan->nvox) * (dtype == PCT_F64 ? 8 : 4);
    if (!disjoint(x, xb, w, L.total)) return PCT_ERR_INVALID_ARG;
    double *proj = reinterpret_cast<double *>(w + L.proj);
    double *q = reinterpret_cast<double *>(w + L.q);
    st = hip_status(launch_fbp_sinogram(f, protons_dev(p), p->n, b, reinterpret_cast<unsigned long long *>(w + L.sum),
                                        reinterpret_cast<unsigned *>(w + L.cnt), proj, nullptr, stream));
    if (st) return st;
    st = hip_status(launch_fbp_filter(f, proj, q, stream));
    if (st) return st;
    return hip_status(launch_fbp_backproject(f, grid_dev(plan->grid), q, x, dtype, stream));
}

const char *pct_status_string(int status)
{
    switch (status) {
    case PCT_OK: return "ok";
    case PCT_ERR_INVALID_ARG: return "invalid argument";
    case PCT_ERR_WORKSPACE: return "workspace missing, too small, misaligned or not uploaded";
    case PCT_ERR_ROW_OVERFLOW: return "traced row longer than max_nnz";
    case PCT_ERR_NONFINITE: return "non-finite input";
    case PCT_ERR_REENTRY: return "voxel re-entry outside the kernel's window";
    case PCT_ERR_HIP: return "HIP runtime error";
    case PCT_ERR_UNSUPPORTED: return "unsupported request";
    case PCT_ERR_CANCELLED: return "stopped on a cancel request";
    default: return "unknown status";
    }
}

int pct_last_hip_error(void) { return g_last_hip_error; }

int pct_profile_read(pct_plan *plan, double ms[2], int64_t launches[2])
{
    if (!plan || !ms || !launches) return PCT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(plan->mu);
    return hip_status(profile_read(*plan, ms, launches));
}

}  // extern "C"
