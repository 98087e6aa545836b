/*
 * FP64 CPU oracle for the proton-CT reconstruction hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * HIP library: every quantity it needs (grid, MLP model constants, proton
 * records) arrives as an argument.
 *
 * What it computes (paper, Section I): the linear system A x = b, with one
 * row a_i of A per proton holding the chord lengths of that proton's most
 * likely path (MLP) through the voxels, b the measured WEPLs and x the
 * relative stopping powers; solved iteratively (Section III) by the block
 * iterative method DROP, one block being the protons processed in parallel
 * (Section IV-B).  The paper cites, but does not print, the MLP and DROP
 * formulas; the readings implemented here are:
 *
 *  MLP  -- the maximum-likelihood path of Schulte et al., Med. Phys. 35:4849
 *          (2008): y_mlp(u1) = (S1^-1 + R1^T S2^-1 R1)^-1 (S1^-1 R0 y0 +
 *          R1^T S2^-1 y2), with the Highland-type scattering matrices S1, S2.
 *          Vertices every `step` mm in depth between fixed tracker planes.
 *  walk -- Siddon's parametric ray/grid intersection (Med. Phys. 12:252,
 *          1985) applied to every polyline segment; voxel of a sub-interval
 *          from its midpoint; half-open voxels; zero-length pieces dropped;
 *          consecutive pieces in the same voxel merged.
 *  row  -- a_ij = sum of the chords with voxel j (re-entries add).  A record
 *          with a non-finite field measures nothing: its row is empty; a row
 *          whose b_i (DROP) or r_i (back projection) is not finite is skipped.
 *  DROP -- block-iterative DROP of Censor, Elfving, Herman & Nikazad (SIAM J.
 *          Sci. Comput. 30:473, 2008) with unit row weights and the diagonal
 *          D = diag(1/s_j), s_j = number of rows of the block that touch j.
 *
 * Everything is FP64, no FMA contraction (build with -ffp-contract=off), and
 * every reduction runs in a fixed order.  FP32 inputs are promoted exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;
    double pitch[3];
    double origin[3];
} orc_grid;

typedef struct {
    double u_in, u_out, step;
    double poly[6];
    double E0, X0;
    int32_t log_term;
} orc_mlp;

typedef struct {
    const float *t_in, *v_in, *th_in, *ph_in, *t_out, *v_out, *th_out, *ph_out, *gantry;
    int64_t n;
} orc_protons;

/* ------------------------------------------------------------------------ */
/* MLP model                                                                 */
/* ------------------------------------------------------------------------ */

/* Number of polyline segments: vertices at depth k*step, k = 0..K-1, plus the
 * exit plane. */
int orc_num_segments(const orc_mlp *m)
{
    double D = m->u_out - m->u_in;
    int K = (int)ceil(D / m->step);
    if (K < 1) K = 1;
    return K;
}

double orc_depth(const orc_mlp *m, int k)
{
    double D = m->u_out - m->u_in;
    double d = k * m->step;
    return d < D ? d : D;
}

static double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
    return r;
}

/* I_m = integral over s in [lo, end] of (end - s)^m P(s) ds, P the
 * 1/(beta^2 p^2) polynomial in depth s [cm].  Substituting w = end - s turns it
 * into the integral over w in [0, end - lo] of w^m P(end - w), and P(end - w)
 * is expanded in powers of w. */
double orc_moment(const orc_mlp *m, int mexp, double lo_cm, double end_cm)
{
    double W = end_cm - lo_cm;
    double sum = 0.0;
    for (int q = 0; q <= 5; q++) {
        /* coefficient of w^q in P(end - w) */
        double cq = 0.0;
        for (int k = q; k <= 5; k++)
            cq += m->poly[k] * binom(k, q) * pow(end_cm, k - q);
        if (q & 1) cq = -cq;
        int p = mexp + q + 1;
        sum += cq * pow(W, p) / p;
    }
    return sum;
}

/* Scattering matrix S(lo -> end) = E0^2 l(end-lo)/X0 * [[I2, I1], [I1, I0]]
 * with l(L) = (1 + 0.038 ln(L/X0))^2 when the log term is on.  Units: cm, rad. */
void orc_sigma(const orc_mlp *m, double lo_cm, double end_cm, double S[3])
{
    double L = end_cm - lo_cm;
    double f = m->E0 * m->E0 / m->X0;
    if (m->log_term) {
        double l = 1.0 + 0.038 * log(L / m->X0);
        f = f * l * l;
    }
    S[0] = f * orc_moment(m, 2, lo_cm, end_cm); /* sigma_t^2      */
    S[1] = f * orc_moment(m, 1, lo_cm, end_cm); /* sigma_t_theta  */
    S[2] = f * orc_moment(m, 0, lo_cm, end_cm); /* sigma_theta^2  */
}

static void mat_inv(const double a[4], double r[4])
{
    double det = a[0] * a[3] - a[1] * a[2];
    r[0] = a[3] / det;
    r[1] = -a[1] / det;
    r[2] = -a[2] / det;
    r[3] = a[0] / det;
}

static void mat_mul(const double a[4], const double b[4], double r[4])
{
    double t0 = a[0] * b[0] + a[1] * b[2];
    double t1 = a[0] * b[1] + a[1] * b[3];
    double t2 = a[2] * b[0] + a[3] * b[2];
    double t3 = a[2] * b[1] + a[3] * b[3];
    r[0] = t0; r[1] = t1; r[2] = t2; r[3] = t3;
}

/* Coefficient table, one row of 4 per vertex k = 0..K:
 *   t_k = c0t*t_in + c0th*th_in + c2t*t_out + c2th*th_out   (t in mm)
 * Rows 0 and K are the measured entry and exit positions.  For interior k,
 * the rows are the first rows of C0 = M S1^-1 R0 and C2 = M R1^T S2^-1 with
 * M = (S1^-1 + R1^T S2^-1 R1)^-1, S1 = S(0 -> d_k), S2 = S(d_k -> D). */
void orc_mlp_table(const orc_mlp *m, double *tab)
{
    int K = orc_num_segments(m);
    double Dcm = (m->u_out - m->u_in) / 10.0;
    tab[0] = 1.0; tab[1] = 0.0; tab[2] = 0.0; tab[3] = 0.0;
    for (int k = 1; k < K; k++) {
        double dcm = orc_depth(m, k) / 10.0;
        double s1[3], s2[3];
        orc_sigma(m, 0.0, dcm, s1);
        orc_sigma(m, dcm, Dcm, s2);
        double S1[4] = {s1[0], s1[1], s1[1], s1[2]};
        double S2[4] = {s2[0], s2[1], s2[1], s2[2]};
        double R0[4] = {1.0, dcm, 0.0, 1.0};
        double R1[4] = {1.0, Dcm - dcm, 0.0, 1.0};
        double R1T[4] = {1.0, 0.0, Dcm - dcm, 1.0};
        double S1i[4], S2i[4], t[4], u[4], Minv[4], M[4], C0[4], C2[4];
        mat_inv(S1, S1i);
        mat_inv(S2, S2i);
        mat_mul(R1T, S2i, t);   /* R1^T S2^-1        */
        mat_mul(t, R1, u);      /* R1^T S2^-1 R1     */
        for (int i = 0; i < 4; i++) Minv[i] = S1i[i] + u[i];
        mat_inv(Minv, M);
        mat_mul(S1i, R0, u);
        mat_mul(M, u, C0);      /* M S1^-1 R0        */
        mat_mul(M, t, C2);      /* M R1^T S2^-1      */
        double *r = tab + 4 * k;
        r[0] = C0[0];
        r[1] = C0[1] * 10.0;    /* cm per unit slope -> mm */
        r[2] = C2[0];
        r[3] = C2[1] * 10.0;
    }
    double *r = tab + 4 * K;
    r[0] = 0.0; r[1] = 0.0; r[2] = 1.0; r[3] = 0.0;
}

/* ------------------------------------------------------------------------ */
/* per-proton path and row                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    double t_in, v_in, th_in, ph_in, t_out, v_out, th_out, ph_out, phi;
} orc_rec;

static orc_rec load_rec(const orc_protons *p, int64_t i)
{
    orc_rec r;
    r.t_in = p->t_in[i];   r.v_in = p->v_in[i];
    r.th_in = p->th_in[i]; r.ph_in = p->ph_in[i];
    r.t_out = p->t_out[i]; r.v_out = p->v_out[i];
    r.th_out = p->th_out[i]; r.ph_out = p->ph_out[i];
    r.phi = p->gantry[i];
    return r;
}

/* Lab coordinates (mm) of vertex k.  Beam frame at gantry angle phi:
 * e_u = (cos, sin, 0), e_t = (-sin, cos, 0), e_v = (0, 0, 1). */
static void vertex(const orc_mlp *m, const double *tab, const orc_rec *r, int k, double P[3])
{
    const double *c = tab + 4 * k;
    double t = c[0] * r->t_in + c[1] * r->th_in + c[2] * r->t_out + c[3] * r->th_out;
    double v = c[0] * r->v_in + c[1] * r->ph_in + c[2] * r->v_out + c[3] * r->ph_out;
    double u = m->u_in + orc_depth(m, k);
    double cs = cos(r->phi), sn = sin(r->phi);
    P[0] = u * cs - t * sn;
    P[1] = u * sn + t * cs;
    P[2] = v;
}

void orc_vertices(const orc_mlp *m, const double *tab, const orc_protons *p, int64_t i, double *P)
{
    orc_rec r = load_rec(p, i);
    int K = orc_num_segments(m);
    for (int k = 0; k <= K; k++) vertex(m, tab, &r, k, P + 3 * k);
}

typedef struct {
    int32_t *vox;
    double *chord;
    int64_t n, cap;
    int32_t last;
} orc_list;

/* Append (j, c) to the emission list, merging with the previous entry when it
 * has the same voxel. */
static void emit(orc_list *L, int32_t j, double c)
{
    if (L->n > 0 && L->last == j) {
        if (L->n <= L->cap) L->chord[L->n - 1] += c;
        return;
    }
    if (L->n < L->cap) {
        L->vox[L->n] = j;
        L->chord[L->n] = c;
    }
    L->last = j;
    L->n++;
}

/* Siddon walk of one straight segment P0 -> P1. */
static void walk_segment(const orc_grid *g, const double P0[3], const double P1[3], orc_list *L)
{
    const int32_t nn[3] = {g->nx, g->ny, g->nz};
    enum { MAXA = 1024 };
    double d[3], alpha[MAXA];
    int na = 0;
    for (int a = 0; a < 3; a++) d[a] = P1[a] - P0[a];
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    alpha[na++] = 0.0;
    alpha[na++] = 1.0;
    for (int a = 0; a < 3; a++) {
        if (d[a] == 0.0) continue;
        double lo = P0[a] < P1[a] ? P0[a] : P1[a];
        double hi = P0[a] < P1[a] ? P1[a] : P0[a];
        /* candidate planes i = 0..n that may lie between the endpoints; the
         * bounds are clamped to [-1, n + 1] in floating point before the cast,
         * so far-away (or non-finite) coordinates never overflow an integer */
        double f0 = floor((lo - g->origin[a]) / g->pitch[a]) - 1.0;
        double f1 = ceil((hi - g->origin[a]) / g->pitch[a]) + 1.0;
        if (!(f0 >= 0.0)) f0 = 0.0;
        if (f0 > nn[a] + 1.0) f0 = nn[a] + 1.0;
        if (!(f1 <= nn[a])) f1 = nn[a];
        if (f1 < -1.0) f1 = -1.0;
        long i0 = (long)f0, i1 = (long)f1;
        for (long i = i0; i <= i1; i++) {
            double plane = g->origin[a] + i * g->pitch[a];
            double al = (plane - P0[a]) / d[a];
            if (al > 0.0 && al < 1.0) {
                if (na == MAXA) abort(); /* a segment crossing > 1000 planes is not a supported input */
                alpha[na++] = al;
            }
        }
    }
    /* insertion sort */
    for (int i = 1; i < na; i++) {
        double v = alpha[i];
        int k = i - 1;
        while (k >= 0 && alpha[k] > v) { alpha[k + 1] = alpha[k]; k--; }
        alpha[k + 1] = v;
    }
    for (int s = 0; s + 1 < na; s++) {
        double a0 = alpha[s], a1 = alpha[s + 1];
        if (!(a1 > a0)) continue;
        double am = 0.5 * (a0 + a1);
        int idx[3], inside = 1;
        for (int a = 0; a < 3; a++) {
            double pm = P0[a] + am * d[a];
            double q = floor((pm - g->origin[a]) / g->pitch[a]);
            if (!(q >= 0.0 && q < nn[a])) { inside = 0; break; }
            idx[a] = (int)q;
        }
        if (!inside) continue;
        int32_t j = idx[0] + g->nx * (idx[1] + g->ny * idx[2]);
        emit(L, j, (a1 - a0) * len);
    }
}

/* ------------------------------------------------------------------------ */
/* Object hull (reading of Section I: the MLP runs between the points where   */
/* the proton enters and leaves the object; the tracks are straight outside). */
/* ------------------------------------------------------------------------ */
static int g_hull = 0;
static double g_hx = 0.0, g_hy = 0.0, g_hr = 0.0;

/* on != 0: hull = z-cylinder (x-cx)^2 + (y-cy)^2 < r^2 (lab mm). */
void orc_set_hull(int on, double cx, double cy, double r)
{
    g_hull = on;
    g_hx = cx;
    g_hy = cy;
    g_hr = r;
}

/* Depth u where the straight track t(u) = t0 + th (u - u0) at gantry angle
 * phi meets the hull circle: the first (smaller) or second root of
 * |(u cos - t sin, u sin + t cos) - c|^2 = r^2.  Returns 0 if it misses. */
static int hull_cross(const orc_rec *r, double t0, double th, double u0, int first, double *u)
{
    double cs = cos(r->phi), sn = sin(r->phi);
    /* point at depth u: (u cs - (t0 + th (u - u0)) sn, u sn + (t0 + th (u - u0)) cs) */
    double px = -(t0 - th * u0) * sn - g_hx, py = (t0 - th * u0) * cs - g_hy;   /* at u = 0 */
    double dx = cs - th * sn, dy = sn + th * cs;                                /* per unit u */
    double A = dx * dx + dy * dy;
    double B = 2.0 * (px * dx + py * dy);
    double C = px * px + py * py - g_hr * g_hr;
    double disc = B * B - 4.0 * A * C;
    if (!(disc > 0.0) || !(A > 0.0)) return 0;
    double sq = sqrt(disc);
    *u = first ? (-B - sq) / (2.0 * A) : (-B + sq) / (2.0 * A);
    return 1;
}

/* Vertices of proton i's polyline into P (3 doubles each, room for `cap`
 * vertices); returns their number.  Without a hull: the K+1 vertices of the
 * shared table.  With a hull: entry tracker point (if the hull entry lies
 * past the entry plane), the MLP from the hull entry to the hull exit with its
 * own table (depth D = hull exit - hull entry, polynomial depth from the hull
 * entry), exit tracker point (if the hull exit lies before the exit plane);
 * a track pair that misses the hull gives the two tracker points. */
int orc_path(const orc_mlp *m, const double *tab, const orc_protons *p, int64_t i, double *P, int cap)
{
    orc_rec r = load_rec(p, i);
    int K = orc_num_segments(m);
    if (!g_hull) {
        if (K + 1 > cap) return -1;
        for (int k = 0; k <= K; k++) vertex(m, tab, &r, k, P + 3 * k);
        return K + 1;
    }
    double cs = cos(r.phi), sn = sin(r.phi);
    double u1, u2;
    int hit = hull_cross(&r, r.t_in, r.th_in, m->u_in, 1, &u1) && hull_cross(&r, r.t_out, r.th_out, m->u_out, 0, &u2);
    if (hit) {
        if (u1 < m->u_in) u1 = m->u_in;
        if (u1 > m->u_out) u1 = m->u_out;
        if (u2 < m->u_in) u2 = m->u_in;
        if (u2 > m->u_out) u2 = m->u_out;
    }
    int n = 0;
    if (!hit || !(u2 > u1)) {
        if (cap < 2) return -1;
        double ts[2] = {r.t_in, r.t_out}, vs[2] = {r.v_in, r.v_out}, us[2] = {m->u_in, m->u_out};
        for (int q = 0; q < 2; q++) {
            P[3 * q] = us[q] * cs - ts[q] * sn;
            P[3 * q + 1] = us[q] * sn + ts[q] * cs;
            P[3 * q + 2] = vs[q];
        }
        return 2;
    }
    /* the sub-problem between the hull crossings, states carried along the tracks */
    orc_mlp m2 = *m;
    m2.u_in = u1;
    m2.u_out = u2;
    orc_rec r2 = r;
    r2.t_in = r.t_in + r.th_in * (u1 - m->u_in);
    r2.v_in = r.v_in + r.ph_in * (u1 - m->u_in);
    r2.t_out = r.t_out + r.th_out * (u2 - m->u_out);
    r2.v_out = r.v_out + r.ph_out * (u2 - m->u_out);
    int K2 = orc_num_segments(&m2);
    if (K2 + 3 > cap) return -1;
    if (u1 > m->u_in) {
        P[0] = m->u_in * cs - r.t_in * sn;
        P[1] = m->u_in * sn + r.t_in * cs;
        P[2] = r.v_in;
        n = 1;
    }
    double *tab2 = (double *)malloc(sizeof(double) * 4 * (K2 + 1));
    orc_mlp_table(&m2, tab2);
    for (int k = 0; k <= K2; k++) vertex(&m2, tab2, &r2, k, P + 3 * (n + k));
    free(tab2);
    n += K2 + 1;
    if (u2 < m->u_out) {
        P[3 * n] = m->u_out * cs - r.t_out * sn;
        P[3 * n + 1] = m->u_out * sn + r.t_out * cs;
        P[3 * n + 2] = r.v_out;
        n++;
    }
    return n;
}

static int rec_finite(const orc_rec *r)
{
    return isfinite(r->t_in) && isfinite(r->v_in) && isfinite(r->th_in) && isfinite(r->ph_in) &&
           isfinite(r->t_out) && isfinite(r->v_out) && isfinite(r->th_out) && isfinite(r->ph_out) &&
           isfinite(r->phi);
}

/* Ordered emission list of proton i.  Returns the full list length; entries
 * beyond `cap` are not written.  A record with a non-finite field is no
 * measurement: its row is empty (length 0). */
int64_t orc_trace(const orc_grid *g, const orc_mlp *m, const double *tab, const orc_protons *p, int64_t i,
                  int64_t cap, int32_t *vox, double *chord)
{
    orc_rec rec = load_rec(p, i);
    if (!rec_finite(&rec)) return 0;
    int K = orc_num_segments(m);
    int vcap = K + 3;
    double *P = (double *)malloc(sizeof(double) * 3 * vcap);
    int nv = orc_path(m, tab, p, i, P, vcap);
    orc_list L = {vox, chord, 0, cap, -1};
    for (int k = 0; k + 1 < nv; k++) walk_segment(g, P + 3 * k, P + 3 * (k + 1), &L);
    free(P);
    return L.n;
}

/* Batched trace: row i written at [i*cap, (i+1)*cap); nnz[i] = full length. */
void orc_trace_batch(const orc_grid *g, const orc_mlp *m, const orc_protons *p, int64_t first, int64_t count,
                     int64_t cap, int32_t *vox, double *chord, int64_t *nnz)
{
    int K = orc_num_segments(m);
    double *tab = (double *)malloc(sizeof(double) * 4 * (K + 1));
    orc_mlp_table(m, tab);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < count; q++)
        nnz[q] = orc_trace(g, m, tab, p, first + q, cap, vox + q * cap, chord + q * cap);
    free(tab);
}

/* Rounding of a chord to a reduced-precision format: first to FP32, then to
 * `bits` significant bits (11 for FP16 with its subnormal floor 2^-24, 8 for
 * BF16), round to nearest, ties to even.  mode: 0 none, 1 fp32, 2 fp16, 3 bf16 */
static double round_sig(double c, int bits, int min_exp)
{
    if (c == 0.0) return 0.0;
    int e;
    frexp(c, &e);                  /* c = f * 2^e, f in [0.5, 1) */
    int q = e - bits;              /* quantum exponent */
    if (q < min_exp) q = min_exp;
    double s = ldexp(c, -q);
    return ldexp(nearbyint(s), q); /* default rounding mode: ties to even */
}

double orc_round_chord(double c, int mode)
{
    if (mode == 0) return c;
    double f = (double)(float)c;
    if (mode == 1) return f;
    if (mode == 2) return round_sig(f, 11, -24);
    return round_sig(f, 8, -149);
}

typedef struct {
    int32_t j;
    int32_t pos; /* position in the emission list */
    double a;
} orc_entry;

static int cmp_entry(const void *x, const void *y)
{
    const orc_entry *a = (const orc_entry *)x, *b = (const orc_entry *)y;
    if (a->j != b->j) return (a->j > b->j) - (a->j < b->j);
    return (a->pos > b->pos) - (a->pos < b->pos);
}

/* Row a_i as distinct voxels in ascending order with a_ij = sum of the chords
 * of voxel j (each chord rounded per `mode` first).  Returns the number of
 * distinct voxels; `rep` (if not NULL) receives the number of non-consecutive
 * repeats (re-entries) in the emission list. */
static int64_t build_row(const orc_grid *g, const orc_mlp *m, const double *tab, const orc_protons *p, int64_t i,
                         int mode, orc_entry **buf, int64_t *bufcap, int64_t *rep)
{
    int64_t cap = 1024;
    int32_t *vox = NULL;
    double *ch = NULL;
    int64_t n;
    for (;;) {
        vox = (int32_t *)realloc(vox, sizeof(int32_t) * cap);
        ch = (double *)realloc(ch, sizeof(double) * cap);
        n = orc_trace(g, m, tab, p, i, cap, vox, ch);
        if (n <= cap) break;
        cap = n;
    }
    if (*bufcap < n) {
        *bufcap = n > 16 ? n : 16;
        *buf = (orc_entry *)realloc(*buf, sizeof(orc_entry) * *bufcap);
    }
    orc_entry *e = *buf;
    for (int64_t q = 0; q < n; q++) {
        e[q].j = vox[q];
        e[q].pos = (int32_t)q;
        e[q].a = orc_round_chord(ch[q], mode);
    }
    free(vox);
    free(ch);
    /* sort by (voxel, emission position), then sum each run of equal voxels in
     * emission order */
    if (n > 1) qsort(e, (size_t)n, sizeof(orc_entry), cmp_entry);   /* an empty row has no buffer */
    int64_t nd = 0;
    for (int64_t q = 0; q < n; q++) {
        if (nd > 0 && e[nd - 1].j == e[q].j) e[nd - 1].a += e[q].a;
        else e[nd++] = e[q];
    }
    /* consecutive repeats were merged at emission, so every remaining
     * duplicate is a re-entry */
    if (rep) *rep = n - nd;
    return nd;
}

/* Distinct-voxel row of proton i (ascending voxel index).  Returns its length. */
int64_t orc_row(const orc_grid *g, const orc_mlp *m, const orc_protons *p, int64_t i, int mode, int64_t cap,
                int32_t *vox, double *a, int64_t *reentries)
{
    int K = orc_num_segments(m);
    double *tab = (double *)malloc(sizeof(double) * 4 * (K + 1));
    orc_mlp_table(m, tab);
    orc_entry *buf = NULL;
    int64_t bc = 0;
    int64_t nd = build_row(g, m, tab, p, i, mode, &buf, &bc, reentries);
    for (int64_t q = 0; q < nd && q < cap; q++) { vox[q] = buf[q].j; a[q] = buf[q].a; }
    free(buf);
    free(tab);
    return nd;
}

/* ------------------------------------------------------------------------ */
/* operators                                                                 */
/* ------------------------------------------------------------------------ */

/* y_i = sum_j a_ij x_j and n2_i = sum_j a_ij^2 (either output may be NULL);
 * nd_i = distinct voxels of row i (may be NULL). */
void orc_forward(const orc_grid *g, const orc_mlp *m, const orc_protons *p, int mode, const double *x, double *y,
                 double *n2, int64_t *nd)
{
    int K = orc_num_segments(m);
    double *tab = (double *)malloc(sizeof(double) * 4 * (K + 1));
    orc_mlp_table(m, tab);
#pragma omp parallel
    {
        orc_entry *buf = NULL;
        int64_t bc = 0;
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < p->n; i++) {
            int64_t n = build_row(g, m, tab, p, i, mode, &buf, &bc, NULL);
            double s = 0.0, q = 0.0;
            for (int64_t k = 0; k < n; k++) {
                if (x) s += buf[k].a * x[buf[k].j];
                q += buf[k].a * buf[k].a;
            }
            if (y) y[i] = s;
            if (n2) n2[i] = q;
            if (nd) nd[i] = n;
        }
        free(buf);
    }
    free(tab);
}

/* g_j += sum_i a_ij r_i, accumulated in proton order (deterministic); a row
 * whose r_i is not finite contributes nothing. */
void orc_backproject(const orc_grid *g, const orc_mlp *m, const orc_protons *p, int mode, const double *r, double *gout)
{
    int K = orc_num_segments(m);
    double *tab = (double *)malloc(sizeof(double) * 4 * (K + 1));
    orc_mlp_table(m, tab);
    const int64_t chunk = 4096;
    orc_entry **rows = (orc_entry **)calloc(chunk, sizeof(orc_entry *));
    int64_t *caps = (int64_t *)calloc(chunk, sizeof(int64_t));
    int64_t *lens = (int64_t *)calloc(chunk, sizeof(int64_t));
    for (int64_t lo = 0; lo < p->n; lo += chunk) {
        int64_t hi = lo + chunk < p->n ? lo + chunk : p->n;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = lo; i < hi; i++)
            lens[i - lo] = build_row(g, m, tab, p, i, mode, &rows[i - lo], &caps[i - lo], NULL);
        for (int64_t i = lo; i < hi; i++) {
            if (!isfinite(r[i])) continue;
            for (int64_t k = 0; k < lens[i - lo]; k++)
                gout[rows[i - lo][k].j] += rows[i - lo][k].a * r[i];
        }
    }
    for (int64_t q = 0; q < chunk; q++) free(rows[q]);
    free(rows); free(caps); free(lens); free(tab);
}

/* Block-iterative DROP.  For every sweep and every block t in
 * [blk_begin, blk_end) (block t = protons [t*B, min(n, (t+1)*B)) in input
 * order):
 *     xbar = x
 *     rho_i = lambda (b_i - a_i . xbar) / ||a_i||^2      (rows with ||a_i|| = 0 skipped)
 *     acc_j = sum_i rho_i a_ij,  s_j = #{i in block : a_ij != entry absent}
 *     x_j = xbar_j + acc_j / s_j                          for s_j > 0
 * A row with a non-finite b_i (or a non-finite record, whose row is empty)
 * is skipped like an empty row: it neither moves x nor counts in s_j.
 * blk_end < 0 means the last block.  Returns the number of blocks run per sweep. */
int64_t orc_drop(const orc_grid *g, const orc_mlp *m, const orc_protons *p, const float *b, double *x,
                 int64_t B, double lambda, int n_iter, int64_t blk_begin, int64_t blk_end, int mode)
{
    int K = orc_num_segments(m);
    double *tab = (double *)malloc(sizeof(double) * 4 * (K + 1));
    orc_mlp_table(m, tab);
    int64_t n = p->n;
    int64_t T = (n + B - 1) / B;
    if (blk_end < 0 || blk_end > T) blk_end = T;
    int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
    double *acc = (double *)calloc(nvox, sizeof(double));
    int64_t *s = (int64_t *)calloc(nvox, sizeof(int64_t));
    orc_entry **rows = (orc_entry **)calloc(B, sizeof(orc_entry *));
    int64_t *caps = (int64_t *)calloc(B, sizeof(int64_t));
    int64_t *lens = (int64_t *)calloc(B, sizeof(int64_t));
    double *rho = (double *)calloc(B, sizeof(double));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * nvox);
    for (int it = 0; it < n_iter; it++) {
        for (int64_t t = blk_begin; t < blk_end; t++) {
            int64_t lo = t * B, hi = lo + B < n ? lo + B : n;
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t i = lo; i < hi; i++) {
                int64_t q = i - lo;
                lens[q] = build_row(g, m, tab, p, i, mode, &rows[q], &caps[q], NULL);
                double dot = 0.0, n2 = 0.0;
                for (int64_t k = 0; k < lens[q]; k++) {
                    dot += rows[q][k].a * x[rows[q][k].j];
                    n2 += rows[q][k].a * rows[q][k].a;
                }
                const double bi = (double)b[i];
                const int use = n2 > 0.0 && isfinite(bi);
                rho[q] = use ? lambda * (bi - dot) / n2 : 0.0;
                if (!use) lens[q] = 0;
            }
            int64_t nt = 0;
            for (int64_t i = lo; i < hi; i++) {
                int64_t q = i - lo;
                for (int64_t k = 0; k < lens[q]; k++) {
                    int32_t j = rows[q][k].j;
                    if (s[j] == 0) touched[nt++] = j;
                    acc[j] += rho[q] * rows[q][k].a;
                    s[j] += 1;
                }
            }
            for (int64_t k = 0; k < nt; k++) {
                int32_t j = touched[k];
                x[j] = x[j] + acc[j] / (double)s[j];
                acc[j] = 0.0;
                s[j] = 0;
            }
        }
    }
    for (int64_t q = 0; q < B; q++) free(rows[q]);
    free(rows); free(caps); free(lens); free(rho); free(touched); free(acc); free(s); free(tab);
    return blk_end - blk_begin;
}

/* ------------------------------------------------------------------------ */
/* total variation (differentiation form)                                    */
/* ------------------------------------------------------------------------ */

/* TV_eps(x) = sum_v sqrt(dx^2 + dy^2 + dz^2 + eps^2), forward differences,
 * difference zero at the last index of each axis.  Returns the value and,
 * if grad != NULL, writes its gradient. */
double orc_tv(const orc_grid *g, const double *x, double eps, double *grad)
{
    int64_t nx = g->nx, ny = g->ny, nz = g->nz;
    int64_t nvox = nx * ny * nz;
    double *sv = (double *)malloc(sizeof(double) * nvox);
    double *dx = (double *)malloc(sizeof(double) * nvox);
    double *dy = (double *)malloc(sizeof(double) * nvox);
    double *dz = (double *)malloc(sizeof(double) * nvox);
    double total = 0.0;
    for (int64_t k = 0; k < nz; k++)
        for (int64_t j = 0; j < ny; j++)
            for (int64_t i = 0; i < nx; i++) {
                int64_t v = i + nx * (j + ny * k);
                dx[v] = i + 1 < nx ? x[v + 1] - x[v] : 0.0;
                dy[v] = j + 1 < ny ? x[v + nx] - x[v] : 0.0;
                dz[v] = k + 1 < nz ? x[v + nx * ny] - x[v] : 0.0;
                sv[v] = sqrt(dx[v] * dx[v] + dy[v] * dy[v] + dz[v] * dz[v] + eps * eps);
                total += sv[v];
            }
    if (grad) {
        for (int64_t k = 0; k < nz; k++)
            for (int64_t j = 0; j < ny; j++)
                for (int64_t i = 0; i < nx; i++) {
                    int64_t v = i + nx * (j + ny * k);
                    double gv = -(dx[v] + dy[v] + dz[v]) / sv[v];
                    if (i > 0) gv += dx[v - 1] / sv[v - 1];
                    if (j > 0) gv += dy[v - nx] / sv[v - nx];
                    if (k > 0) gv += dz[v - nx * ny] / sv[v - nx * ny];
                    grad[v] = gv;
                }
    }
    free(sv); free(dx); free(dy); free(dz);
    return total;
}
