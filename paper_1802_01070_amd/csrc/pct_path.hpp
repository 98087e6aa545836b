// Device-side path machinery: MLP vertices from the coefficient table, the
// per-segment voxel walk, consecutive-piece merging and the voxel re-entry
// tracker that turns the piece stream into matrix-row semantics.
//
// Geometry is evaluated in FP64: on CDNA4 the vector FP64 FMA/add/mul rate
// equals the (unpacked) FP32 rate, and FP64 keeps every plane-crossing
// decision identical to an FP64 reference except on measure-zero ties.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pct_internal.h"

namespace pct {

struct Rec {
    double t_in, v_in, th_in, ph_in, t_out, v_out, th_out, ph_out;
    double cs, sn;  // cos, sin of the gantry angle
};

__device__ __forceinline__ Rec load_rec(const ProtonsDev &p, int64_t i)
{
    Rec r;
    r.t_in = p.t_in[i];
    r.v_in = p.v_in[i];
    r.th_in = p.th_in[i];
    r.ph_in = p.ph_in[i];
    r.t_out = p.t_out[i];
    r.v_out = p.v_out[i];
    r.th_out = p.th_out[i];
    r.ph_out = p.ph_out[i];
    double phi = p.gantry[i];
    sincos(phi, &r.sn, &r.cs);
    return r;
}

__device__ __forceinline__ bool rec_finite(const Rec &r)
{
    return isfinite(r.t_in) && isfinite(r.v_in) && isfinite(r.th_in) && isfinite(r.ph_in) &&
           isfinite(r.t_out) && isfinite(r.v_out) && isfinite(r.th_out) && isfinite(r.ph_out) &&
           isfinite(r.cs) && isfinite(r.sn);
}

// Vertex k of the most likely path in lab coordinates (mm).  Row k of the
// table gives t_k = c0t t_in + c0th th_in + c2t t_out + c2th th_out (same for
// v) and the depth coordinate u_k.
__device__ __forceinline__ void vertex(const Rec &r, const double *__restrict__ row, double P[3])
{
    const double c0t = row[0], c0h = row[1], c2t = row[2], c2h = row[3], u = row[4];
    double t = c0t * r.t_in + c0h * r.th_in + c2t * r.t_out + c2h * r.th_out;
    double v = c0t * r.v_in + c0h * r.ph_in + c2t * r.v_out + c2h * r.ph_out;
    P[0] = u * r.cs - t * r.sn;
    P[1] = u * r.sn + t * r.cs;
    P[2] = v;
}

// Walk of one straight segment P0 -> P1 through the part of the grid whose
// index along axis `ra` lies in [r_lo, r_hi] (Siddon's parametrisation
// P0 + alpha (P1 - P0), alpha in [0, 1]).  Calls sink.piece(ix, iy, iz, chord)
// for every sub-interval of positive length inside that box, in path order.
// The box faces along `ra` are grid planes, so the pieces are exactly the
// pieces of the full walk that fall in the index range.  Indices handed to
// the sink are always inside the grid.
template <class Sink>
__device__ __forceinline__ void walk_segment_range(const double P0[3], const double P1[3], const GridDev &g,
                                                   int ra, int r_lo, int r_hi, Sink &sink)
{
    double d[3], inv[3], lo[3], hi[3];
    int ilo[3], ihi[3];
    double a_lo = 0.0, a_hi = 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a == ra) {
            ilo[a] = r_lo;
            ihi[a] = r_hi;
            lo[a] = g.lo[a] + r_lo * g.pitch[a];
            hi[a] = g.lo[a] + (r_hi + 1) * g.pitch[a];
        } else {
            ilo[a] = 0;
            ihi[a] = g.n[a] - 1;
            lo[a] = g.lo[a];
            hi[a] = g.hi[a];
        }
        d[a] = P1[a] - P0[a];
        if (d[a] != 0.0) {
            inv[a] = 1.0 / d[a];
            double t0 = (lo[a] - P0[a]) * inv[a];
            double t1 = (hi[a] - P0[a]) * inv[a];
            a_lo = fmax(a_lo, fmin(t0, t1));
            // d * inv is the parameter a plane through the end point gets
            // below; it may round under 1, and the walk must stop there, not
            // step into the next voxel for a piece of rounding length
            a_hi = fmin(a_hi, fmin(fmax(t0, t1), d[a] * inv[a]));
        } else {
            inv[a] = 0.0;
            if (!(P0[a] >= lo[a] && P0[a] < hi[a])) a_hi = -1.0;
        }
    }
    if (!(a_lo < a_hi)) return;  // also rejects NaN
    const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);

    int idx[3], stp[3];
    double anext[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double pos = P0[a] + a_lo * d[a];
        double q = (pos - g.lo[a]) * g.inv_pitch[a];
        double f = floor(q);
        int i = int(fmin(fmax(f, -1.0), double(g.n[a])));
        if (d[a] < 0.0 && f == q) i -= 1;  // on a plane and moving down
        i = min(max(i, ilo[a]), ihi[a]);
        idx[a] = i;
        if (d[a] > 0.0) {
            stp[a] = 1;
            anext[a] = (g.lo[a] + (i + 1) * g.pitch[a] - P0[a]) * inv[a];
        } else if (d[a] < 0.0) {
            stp[a] = -1;
            anext[a] = (g.lo[a] + i * g.pitch[a] - P0[a]) * inv[a];
        } else {
            stp[a] = 0;
            anext[a] = 2.0;
        }
    }
    double acur = a_lo;
    const int max_it = g.n[0] + g.n[1] + g.n[2] + 4;
    for (int it = 0; it < max_it; ++it) {
        double am = fmin(fmin(anext[0], anext[1]), anext[2]);
        double aend = fmin(am, a_hi);
        if (aend > acur) sink.piece(idx[0], idx[1], idx[2], (aend - acur) * len);
        if (!(am < a_hi)) break;
        bool out = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (anext[a] == am) {
                int i = idx[a] + stp[a];
                out |= (i < ilo[a]) | (i > ihi[a]);
                idx[a] = i;
                anext[a] = (g.lo[a] + (i + (stp[a] > 0 ? 1 : 0)) * g.pitch[a] - P0[a]) * inv[a];
            }
        }
        if (out) break;
        acur = fmax(acur, am);
    }
}

template <class Sink>
__device__ __forceinline__ void walk_segment(const double P0[3], const double P1[3], const GridDev &g, Sink &sink)
{
    walk_segment_range(P0, P1, g, 0, 0, g.n[0] - 1, sink);
}

// ---------------------------------------------------------------------------
// Per-proton polyline
// ---------------------------------------------------------------------------
// Coefficients of one interior MLP vertex at depth d (mm) of a path of depth D
// (mm), row layout of the shared table: c0t, c0th (mm), c2t, c2th (mm).  The
// same mathematics as the host table: scattering matrices by 4-point
// Gauss-Legendre (exact for the degree-7 integrands) and the Kalman-gain form
// of the conditional mean, depth of the polynomial measured from the start of
// the path.
__device__ __forceinline__ double mlp_poly(const PathSrc &m, double s)
{
    double v = 0.0;
    for (int k = 5; k >= 0; --k) v = v * s + m.poly[k];
    return v;
}

__device__ __forceinline__ void mlp_scatter(const PathSrc &m, double lo, double end, double S[4])
{
    const double r1 = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
    const double r2 = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
    const double w1 = (18.0 + sqrt(30.0)) / 36.0;
    const double w2 = (18.0 - sqrt(30.0)) / 36.0;
    const double xs[4] = {-r2, -r1, r1, r2};
    const double ws[4] = {w2, w1, w1, w2};
    const double h = 0.5 * (end - lo), c = 0.5 * (end + lo);
    double J0 = 0.0, J1 = 0.0, J2 = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double s = c + h * xs[i];
        const double w = ws[i] * h * mlp_poly(m, s);
        const double e = end - s;
        J0 += w;
        J1 += w * e;
        J2 += w * e * e;
    }
    double f = m.E0 * m.E0 / m.X0;
    if (m.log_term) {
        const double l = 1.0 + 0.038 * log((end - lo) / m.X0);
        f *= l * l;
    }
    S[0] = f * J2;
    S[1] = f * J1;
    S[2] = f * J1;
    S[3] = f * J0;
}

__device__ __forceinline__ void mlp_coeffs(const PathSrc &m, double d_mm, double D_mm, double c[4])
{
    const double d = d_mm / 10.0, Dcm = D_mm / 10.0;
    double S1[4], S2[4];
    mlp_scatter(m, 0.0, d, S1);
    mlp_scatter(m, d, Dcm, S2);
    const double e = Dcm - d;
    const double a = S1[0] + 2.0 * e * S1[1] + e * e * S1[3] + S2[0];
    const double bb = S1[1] + e * S1[3] + S2[1];
    const double dd = S1[3] + S2[3];
    const double det = a * dd - bb * bb;
    const double Ti[4] = {dd / det, -bb / det, -bb / det, a / det};
    const double U[4] = {S1[0] + e * S1[1], S1[1], S1[2] + e * S1[3], S1[3]};
    const double G0 = U[0] * Ti[0] + U[1] * Ti[2];
    const double G1 = U[0] * Ti[1] + U[1] * Ti[3];
    const double q0 = 1.0 - G0;
    const double q1 = -G0 * e - G1;
    c[0] = q0;
    c[1] = (q0 * d + q1) * 10.0;
    c[2] = G0;
    c[3] = G1 * 10.0;
}

// Where a straight track t(u) = t0 + th (u - u0) of gantry angle (cs, sn)
// crosses the hull circle: the smaller (first = true) or larger root in u.
__device__ __forceinline__ bool hull_cross(const PathSrc &m, const Rec &r, double t0, double th, double u0,
                                           bool first, double &u)
{
    const double ct = t0 - th * u0;  // t at u = 0
    const double a1 = r.cs - th * r.sn, b1 = r.sn + th * r.cs;
    const double a0 = -ct * r.sn - m.hx, b0 = ct * r.cs - m.hy;
    const double A = a1 * a1 + b1 * b1;
    const double B = a1 * a0 + b1 * b0;
    const double C = a0 * a0 + b0 * b0 - m.hr * m.hr;
    const double disc = B * B - A * C;
    if (!(disc > 0.0) || !(A > 0.0)) return false;
    const double q = -(B + copysign(sqrt(disc), B));
    double x1 = q / A, x2 = C / q;
    if (q == 0.0) x1 = x2 = -B / A;
    u = first ? fmin(x1, x2) : fmax(x1, x2);
    return true;
}

struct PathState {
    int nv;         // vertices
    int pre, kh;    // leading tracker vertex (0/1), MLP segments inside the hull
    bool miss;      // the tracks do not reach the hull: one straight segment
    double uh_in, uh_out, t0, v0, t1, v1;
};

// The hull path is a separate instantiation of the kernels (template flag
// HULL), so the table path keeps its register allocation.
__device__ __forceinline__ PathState hull_prepare(const Rec &r, const PathSrc &m)
{
    PathState ps{};
    double u1 = 0.0, u2 = 0.0;
    const bool hit = hull_cross(m, r, r.t_in, r.th_in, m.u_in, true, u1) &&
                     hull_cross(m, r, r.t_out, r.th_out, m.u_out, false, u2);
    ps.uh_in = fmin(fmax(u1, m.u_in), m.u_out);
    ps.uh_out = fmin(fmax(u2, m.u_in), m.u_out);
    if (!hit || !(ps.uh_out > ps.uh_in)) {
        ps.miss = true;
        ps.nv = 2;
        return ps;
    }
    const double D = ps.uh_out - ps.uh_in;
    ps.kh = max(1, int(ceil(D / m.step)));
    ps.pre = ps.uh_in > m.u_in ? 1 : 0;
    const int post = ps.uh_out < m.u_out ? 1 : 0;
    ps.nv = ps.pre + ps.kh + 1 + post;
    ps.t0 = r.t_in + r.th_in * (ps.uh_in - m.u_in);
    ps.v0 = r.v_in + r.ph_in * (ps.uh_in - m.u_in);
    ps.t1 = r.t_out + r.th_out * (ps.uh_out - m.u_out);
    ps.v1 = r.v_out + r.ph_out * (ps.uh_out - m.u_out);
    return ps;
}

template <bool HULL>
__device__ __forceinline__ PathState path_prepare(const Rec &r, const PathSrc &m)
{
    if constexpr (HULL) {
        return hull_prepare(r, m);
    } else {
        PathState ps{};
        ps.nv = m.K + 1;
        return ps;
    }
}

__device__ __forceinline__ void hull_vertex(const Rec &r, const PathSrc &m, const PathState &ps, int k, double *P)
{
    double u, t, v;
    const int j = k - ps.pre;
    if (ps.miss) {
        u = k == 0 ? m.u_in : m.u_out;
        t = k == 0 ? r.t_in : r.t_out;
        v = k == 0 ? r.v_in : r.v_out;
    } else if (j < 0) {
        u = m.u_in;
        t = r.t_in;
        v = r.v_in;
    } else if (j > ps.kh) {
        u = m.u_out;
        t = r.t_out;
        v = r.v_out;
    } else if (j == 0) {
        u = ps.uh_in;
        t = ps.t0;
        v = ps.v0;
    } else if (j == ps.kh) {
        u = ps.uh_out;
        t = ps.t1;
        v = ps.v1;
    } else {
        const double d = j * m.step;
        double c[4];
        mlp_coeffs(m, d, ps.uh_out - ps.uh_in, c);
        u = ps.uh_in + d;
        t = c[0] * ps.t0 + c[1] * r.th_in + c[2] * ps.t1 + c[3] * r.th_out;
        v = c[0] * ps.v0 + c[1] * r.ph_in + c[2] * ps.v1 + c[3] * r.ph_out;
    }
    P[0] = u * r.cs - t * r.sn;
    P[1] = u * r.sn + t * r.cs;
    P[2] = v;
}

// Vertex k (0 <= k < ps.nv) in lab coordinates (mm).
template <bool HULL>
__device__ __forceinline__ void path_vertex(const Rec &r, const PathSrc &m, const PathState &ps, int k, double P[3])
{
    if constexpr (HULL)
        hull_vertex(r, m, ps, k, P);
    else
        vertex(r, m.tab + k * kRowDoubles, P);
}

// Walk of the whole polyline of one proton.
template <bool HULL, class Sink>
__device__ __forceinline__ void walk_path(const Rec &r, const PathSrc &src, const GridDev &g, Sink &sink)
{
    const PathState ps = path_prepare<HULL>(r, src);
    double P0[3], P1[3];
    path_vertex<HULL>(r, src, ps, 0, P0);
    for (int k = 1; k < ps.nv; ++k) {
        path_vertex<HULL>(r, src, ps, k, P1);
        sink.segment(P1[0] - P0[0], P1[1] - P0[1]);
        walk_segment(P0, P1, g, sink);
        P0[0] = P1[0];
        P0[1] = P1[1];
        P0[2] = P1[2];
    }
}

// Rounding of a chord to the solver's chord format: FP64 -> FP32 (RNE), then
// to FP16 or BF16 (RNE).  The second step works on the FP32 bit pattern: a
// plain half(float(c)) may be folded by the compiler into one direct
// FP64 -> FP16 rounding, which differs from the two-step rounding on FP16 ties.
template <int CHORD>
__device__ __forceinline__ double round_chord(double c)
{
    if constexpr (CHORD == PCT_CHORD_F64) {
        return c;
    } else {
        float f = float(c);
        if constexpr (CHORD == PCT_CHORD_F32) {
            return double(f);
        } else if constexpr (CHORD == PCT_CHORD_F16) {
            if (fabsf(f) < 0x1p-14f) {
                // FP16 subnormal range: fixed quantum 2^-24 (scaling by powers of
                // two is exact; rintf rounds to nearest even)
                return double(rintf(f * 0x1p24f) * 0x1p-24f);
            }
            uint32_t u = __float_as_uint(f);
            u = (u + 0x0FFFu + ((u >> 13) & 1u)) & 0xFFFFE000u;  // keep 10 mantissa bits
            return double(fminf(__uint_as_float(u), 65504.0f));
        } else {
            uint32_t u = __float_as_uint(f);
            u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
            return double(__uint_as_float(u));
        }
    }
}

// Re-entry tracker.  A voxel can be visited again only while the path stays in
// one slab of the dominant in-plane axis (the path is monotone along it), and
// only after the index along one of the two other axes has reversed direction
// inside that slab.  Until such a reversal every merged piece is a first visit;
// afterwards pieces are looked up in a register window of the last R pieces.
// If the window cannot cover the slab, or the path is not monotone along the
// dominant axis, the proton is flagged (PCT_DEV_REENTRY).
struct Reentry {
    static constexpr int R = 4;
    int dom;      // 0: x dominant, 1: y dominant
    int dsign;    // direction of travel along the dominant axis
    int cur_a, prev_b, prev_z, sgn_b, sgn_z, nslab;
    bool rev, unsafe;
    int rj[R];
    double rc[R];

    __device__ __forceinline__ void init(const Rec &r)
    {
        dom = fabs(r.cs) >= fabs(r.sn) ? 0 : 1;
        double e = dom == 0 ? r.cs : r.sn;
        dsign = e > 0.0 ? 1 : -1;
        cur_a = -1;
        prev_b = prev_z = 0;
        sgn_b = sgn_z = 0;
        nslab = 0;
        rev = false;
        unsafe = false;
#pragma unroll
        for (int s = 0; s < R; ++s) {
            rj[s] = -1;
            rc[s] = 0.0;
        }
    }

    __device__ __forceinline__ void segment(double dx, double dy)
    {
        double da = dom == 0 ? dx : dy;
        if (!(da * dsign > 0.0)) unsafe = true;
    }

    // Registers merged piece (j, c); returns the sum of the chords of earlier
    // pieces with the same voxel (0 on a first visit) and sets `first`.
    __device__ __forceinline__ double visit(int j, int ix, int iy, int iz, double c, bool &first)
    {
        int ia = dom == 0 ? ix : iy;
        int ib = dom == 0 ? iy : ix;
        if (ia != cur_a) {
            cur_a = ia;
            sgn_b = sgn_z = 0;
            rev = false;
            nslab = 0;
        } else {
            int db = ib - prev_b, dz = iz - prev_z;
            if (db != 0) {
                int s = db > 0 ? 1 : -1;
                if (sgn_b == 0) sgn_b = s;
                else if (sgn_b != s) rev = true;
            }
            if (dz != 0) {
                int s = dz > 0 ? 1 : -1;
                if (sgn_z == 0) sgn_z = s;
                else if (sgn_z != s) rev = true;
            }
        }
        prev_b = ib;
        prev_z = iz;
        double aprev = 0.0;
        first = true;
        if (rev) {
            if (nslab > R) unsafe = true;
#pragma unroll
            for (int s = 0; s < R; ++s) {
                if (rj[s] == j) {
                    aprev += rc[s];
                    first = false;
                }
            }
        }
#pragma unroll
        for (int s = R - 1; s > 0; --s) {
            rj[s] = rj[s - 1];
            rc[s] = rc[s - 1];
        }
        rj[0] = j;
        rc[0] = c;
        ++nslab;
        return aprev;
    }
};

}  // namespace pct
