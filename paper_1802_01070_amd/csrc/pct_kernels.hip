// HIP kernels of the reconstruction path for gfx950 and their launchers.
//
//   k_trace        ordered emission list of each proton's path (debug/parity)
//   k_forward      y = A x, ||a_i||^2   (one lane per proton, gathers)
//   k_backproject  g += A^T r           (one lane per proton, LDS-summed, atomics)
//   k_drop_block   DROP block, LPP lanes per proton: walk -> a_i.x, ||a_i||^2 ->
//                  rho_i -> re-walk and scatter rho_i a_ij into the block
//                  accumulator and the per-voxel row count; records the
//                  block's touched voxel index range
//   k_drop_rows    the same with one lane per proton (very long paths)
//   k_drop_commit  x_j += acc_j / s_j over the touched range, reset
//   k_tv           smoothed total variation value and gradient
#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "pct_internal.h"
#include "pct_path.hpp"

namespace pct {

constexpr int kWG = 256;

__device__ __forceinline__ void raise_status(unsigned *status, unsigned bit)
{
    atomicOr(status, bit);
}

// Block-boundary gate of a cancellable DROP call (workspace header words).
// Every per-block kernel returns at once while the gate is closed; the last
// workgroup of each commit launch counts the block step and, when the host
// has requested a stop, closes the gate for the launches after it.  The
// gate word changes only there, after every workgroup of that launch has
// read it, so all workgroups of a launch take the same decision.
struct GateDev {
    int *halt;          // nullptr: the call is not cancellable
    unsigned *wg_done;  // workgroups of the running commit launch that ended
    const int *cancel;  // the host's request
    long long *done;    // block steps applied by the call
    unsigned *status;
};

__device__ __forceinline__ bool gate_closed(const int *halt) { return halt && *halt != 0; }

__device__ __forceinline__ void gate_commit_end(const GateDev &gt)
{
    if (!gt.halt) return;
    // every wave of the workgroup has read the gate (a load consumed by the
    // entry branch) before the workgroup is counted
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned k = atomicAdd(gt.wg_done, 1u);
        if (k == gridDim.x - 1) {
            *gt.wg_done = 0u;
            *gt.done += 1;
            if (__hip_atomic_load(gt.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0) {
                *gt.halt = 1;
                atomicOr(gt.status, PCT_DEV_CANCELLED);
            }
        }
    }
}

// Start of a cancellable call: gate open, no block step applied.
__global__ void k_gate_begin(GateDev gt)
{
    if (threadIdx.x == 0) {
        *gt.halt = 0;
        *gt.wg_done = 0u;
        *gt.done = 0;
    }
}

// Merges consecutive pieces in the same voxel and hands merged pieces (with
// the chord rounded to the solver's format) to Inner::final.
template <class Inner, int CHORD>
struct Merge {
    Inner &in;
    int nx, ny;
    int cj, cx, cy, cz;
    double cc;

    __device__ __forceinline__ Merge(Inner &inner, const GridDev &grid)
        : in(inner), nx(grid.n[0]), ny(grid.n[1]), cj(-1), cx(0), cy(0), cz(0), cc(0.0)
    {
    }

    __device__ __forceinline__ void segment(double dx, double dy) { in.segment(dx, dy); }

    __device__ __forceinline__ void piece(int ix, int iy, int iz, double c)
    {
        int j = ix + nx * (iy + ny * iz);
        if (j == cj) {
            cc += c;
            return;
        }
        if (cj >= 0) in.final(cj, cx, cy, cz, round_chord<CHORD>(cc));
        cj = j;
        cx = ix;
        cy = iy;
        cz = iz;
        cc = c;
    }

    __device__ __forceinline__ void finish()
    {
        if (cj >= 0) in.final(cj, cx, cy, cz, round_chord<CHORD>(cc));
        cj = -1;
    }
};

// ---------------------------------------------------------------------------
// trace
// ---------------------------------------------------------------------------
struct TraceSink {
    int32_t *vox;
    double *chord;
    int32_t cap, n;
    __device__ __forceinline__ void segment(double, double) {}
    __device__ __forceinline__ void final(int j, int, int, int, double c)
    {
        if (n < cap) {
            vox[n] = j;
            chord[n] = c;
        }
        ++n;
    }
};

template <bool HULL>
__global__ void __launch_bounds__(kWG) k_trace(ProtonsDev p, int64_t first, int64_t count, int32_t max_nnz,
                                               int32_t *vox, double *chord, int32_t *nnz,
                                               const PathSrc src,  GridDev g, unsigned *status)
{
    int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= count) return;
    Rec r = load_rec(p, first + q);
    TraceSink ts{vox + q * max_nnz, chord + q * max_nnz, max_nnz, 0};
    if (rec_finite(r)) {
        Merge<TraceSink, PCT_CHORD_F64> m(ts, g);
        walk_path<HULL>(r, src, g, m);
        m.finish();
    } else {
        raise_status(status, PCT_DEV_NONFINITE);
    }
    nnz[q] = ts.n;
    if (ts.n > max_nnz) raise_status(status, PCT_DEV_ROW_OVERFLOW);
}

// ---------------------------------------------------------------------------
// forward projection
// ---------------------------------------------------------------------------
// Value of the iterate at voxel j seen by a block.
template <typename T>
struct PlainX {
    const T *__restrict__ x;
    __device__ __forceinline__ double operator()(int j) const { return double(x[j]); }
};

template <typename T, class XA = PlainX<T>>
struct DotSink {
    XA x;
    Reentry re;
    double dot, n2;
    __device__ __forceinline__ void segment(double dx, double dy) { re.segment(dx, dy); }
    __device__ __forceinline__ void final(int j, int ix, int iy, int iz, double c)
    {
        bool first;
        double aprev = re.visit(j, ix, iy, iz, c, first);
        dot += c * x(j);
        n2 += c * (2.0 * aprev + c);
    }
};

template <typename T, bool HULL>
__global__ void __launch_bounds__(kWG) k_forward(ProtonsDev p, int64_t first, int64_t n, const T *__restrict__ x,
                                                 T *y, T *nrm2, const PathSrc src, GridDev g, unsigned *status)
{
    int64_t i = first + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Rec r = load_rec(p, i);
    DotSink<T> s;
    s.x = PlainX<T>{x};
    s.dot = 0.0;
    s.n2 = 0.0;
    s.re.init(r);
    if (rec_finite(r)) {
        Merge<DotSink<T>, PCT_CHORD_F64> m(s, g);
        walk_path<HULL>(r, src, g, m);
        m.finish();
        if (s.re.unsafe) raise_status(status, PCT_DEV_REENTRY);
    } else {
        raise_status(status, PCT_DEV_NONFINITE);
    }
    y[i] = T(s.dot);
    if (nrm2) nrm2[i] = T(s.n2);
}

// ---------------------------------------------------------------------------
// back projection
// ---------------------------------------------------------------------------
// Back projection g += A^T r, one lane per proton.  The 256 rows of a
// workgroup are consecutive in the scan, and an angle-sorted scan's
// consecutive rows cross nearly the same voxels, so the workgroup first sums
// its pieces in an LDS table keyed by voxel (open addressing, a few probes)
// and each distinct voxel then reaches HBM with one atomic.  A piece that
// finds no slot goes straight to HBM, and so do the later pieces of its lane
// (the table is filling up: an unsorted scan).
template <typename T>
struct BpTable {
    static constexpr int kSlots = sizeof(T) == 4 ? 8192 : 4096;  // 64 KB / 48 KB of LDS
    static constexpr int kBits = sizeof(T) == 4 ? 13 : 12;
    static constexpr int kProbes = 8;
};

template <typename T>
struct HashScatterSink {
    int *keys;
    T *vals;
    T *g;
    double r;
    bool full;  // a probe sequence of this lane found no slot
    __device__ __forceinline__ void segment(double, double) {}
    __device__ __forceinline__ void final(int j, int, int, int, double c)
    {
        using B = BpTable<T>;
        const T v = T(r * c);
        if (!full) {
            unsigned s = (unsigned(j) * 2654435761u) >> (32 - B::kBits);
            for (int q = 0; q < B::kProbes; ++q) {
                int k = *reinterpret_cast<volatile int *>(keys + s);
                if (k == -1) {
                    const int old = atomicCAS(keys + s, -1, j);
                    k = old == -1 ? j : old;
                }
                if (k == j) {
                    atomicAdd(vals + s, v);
                    return;
                }
                s = (s + 1) & (B::kSlots - 1);
            }
            full = true;
        }
        atomicAdd(g + j, v);
    }
};

template <typename T, bool HULL>
__global__ void __launch_bounds__(kWG) k_backproject(ProtonsDev p, int64_t first, int64_t n,
                                                     const T *__restrict__ rv, T *gout, const PathSrc src, GridDev g,
                                                     unsigned *status)
{
    using B = BpTable<T>;
    __shared__ int keys[B::kSlots];
    __shared__ T vals[B::kSlots];
    for (int q = threadIdx.x; q < B::kSlots; q += kWG) {
        keys[q] = -1;
        vals[q] = T(0);
    }
    __syncthreads();
    const int64_t i = first + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    bool active = i < n;
    double ri = 0.0;
    Rec r{};
    if (active) {
        ri = double(rv[i]);
        if (ri == 0.0) {
            active = false;
        } else {
            r = load_rec(p, i);
            if (!rec_finite(r) || !isfinite(ri)) {
                raise_status(status, PCT_DEV_NONFINITE);
                active = false;
            }
        }
    }
    if (active) {
        HashScatterSink<T> s{keys, vals, gout, ri, false};
        Merge<HashScatterSink<T>, PCT_CHORD_F64> m(s, g);
        walk_path<HULL>(r, src, g, m);
        m.finish();
    }
    __syncthreads();
    for (int q = threadIdx.x; q < B::kSlots; q += kWG) {
        const int k = keys[q];
        if (k >= 0) atomicAdd(gout + k, vals[q]);
    }
}

// ---------------------------------------------------------------------------
// DROP
// ---------------------------------------------------------------------------
// Block accumulator for the FP32 value type: one 64-bit word per voxel holding
// the number of block rows that touch the voxel (bits 63..44) and the sum of
// rho_i a_ij in fixed point with kFixBits fractional bits (two's complement in
// the low bits).  One integer add per piece updates both, and integer
// addition makes the block sum independent of the order of the adds.  The sum
// must stay below kSumMax = 2^(43 - kFixBits) in magnitude.  A contribution of
// kFixMax or more is clamped to it and raises PCT_DEV_ACC_RANGE, a NaN one
// counts as zero.  The binned schedule also bounds every voxel's block sum by
// the sum over the block's rows of their largest contribution and raises the
// bit when that bound reaches kSumMax.
constexpr int kFixBits = 28;
constexpr int kCntShift = 44;
constexpr double kFixScale = double(1u << kFixBits);
constexpr double kFixMax = double(1u << 12);
constexpr double kSumMax = double(1ull << (kCntShift - 1 - kFixBits));

__device__ __forceinline__ unsigned long long pack_contribution(double v, bool first, unsigned *status)
{
    if (!(fabs(v) < kFixMax)) {
        atomicOr(status, PCT_DEV_ACC_RANGE);
        if (v != v) v = 0.0;
        else v = fmin(fmax(v, -kFixMax), kFixMax);
    }
    const long long q = llrint(v * kFixScale);
    return static_cast<unsigned long long>(q) + (first ? (1ull << kCntShift) : 0ull);
}

__device__ __forceinline__ void unpack_accumulator(unsigned long long w, int &cnt, double &sum)
{
    const long long W = static_cast<long long>(w);
    const long long c = (W + (1ll << (kCntShift - 1))) >> kCntShift;
    const long long V = W - (c << kCntShift);
    cnt = int(c);
    sum = double(V) * (1.0 / kFixScale);
}

// Order-independent FP64 block sums (deterministic mode): each contribution
// v is split into hi = round(v 2^28) and lo = round((v - hi 2^-28) 2^72), the
// first part exact (v's bits above 2^-28), the second within 2^-73, and both
// are summed in 64-bit integers, so the block sum hi 2^-28 + lo 2^-72 does not
// depend on the order of the adds.  A contribution of 2^16 or more (NaN: 0)
// is clamped and raises PCT_DEV_ACC_RANGE, which keeps the sums of blocks
// below 2^19 rows inside 64 bits.
constexpr double kDetHiScale = 268435456.0;                 // 2^28
constexpr double kDetLoScale = 4722366482869645213696.0;    // 2^72
constexpr double kDetMax = 65536.0;                         // 2^16

__device__ __forceinline__ void det_add(long long *hi, long long *lo, int j, double v, unsigned *status)
{
    if (!(fabs(v) < kDetMax)) {
        atomicOr(status, PCT_DEV_ACC_RANGE);
        v = v != v ? 0.0 : fmin(fmax(v, -kDetMax), kDetMax);
    }
    const double qh = rint(v * kDetHiScale);
    const double r = v - qh * (1.0 / kDetHiScale);
    atomicAdd(reinterpret_cast<unsigned long long *>(hi) + j, static_cast<unsigned long long>(static_cast<long long>(qh)));
    atomicAdd(reinterpret_cast<unsigned long long *>(lo) + j, static_cast<unsigned long long>(llrint(r * kDetLoScale)));
}

__device__ __forceinline__ double det_sum(long long hi, long long lo)
{
    return double(hi) * (1.0 / kDetHiScale) + double(lo) * (1.0 / kDetLoScale);
}

// One piece of a row into the block's accumulation: FP32 packed word; FP64
// double atomic, or the integer pair when acc_lo is given; the row count once.
template <typename T>
__device__ __forceinline__ void scatter_one(void *acc, long long *acc_lo, int32_t *cnt, int j, double v, bool first,
                                            unsigned *status)
{
    if constexpr (sizeof(T) == 4) {
        atomicAdd(static_cast<unsigned long long *>(acc) + j, pack_contribution(v, first, status));
    } else {
        if (acc_lo)
            det_add(static_cast<long long *>(acc), acc_lo, j, v, status);
        else
            atomicAdd(static_cast<double *>(acc) + j, v);
        if (first) atomicAdd(cnt + j, 1);
    }
}

// Scatter of one row: acc_j += rho a_ij and s_j += 1 once per row.  FP32 value
// type: packed 64-bit accumulator; FP64: double accumulator (or the integer
// pair) plus int count.
template <typename T>
struct DropScatterSink {
    void *acc;
    long long *acc_lo = nullptr;  // FP64 deterministic mode: low words of the integer pair
    int32_t *cnt;
    unsigned *status;
    Reentry re;
    double rho;
    int jmin, jmax;
    __device__ __forceinline__ void segment(double dx, double dy) { re.segment(dx, dy); }
    __device__ __forceinline__ void final(int j, int ix, int iy, int iz, double c)
    {
        bool first;
        re.visit(j, ix, iy, iz, c, first);
        scatter_one<T>(acc, acc_lo, cnt, j, rho * c, first, status);
        jmin = min(jmin, j);
        jmax = max(jmax, j);
    }
};

// Workgroup-wide min/max of the touched voxel range, then one atomic pair per
// workgroup into the block's range words.  Every thread of the workgroup must
// call it.
__device__ __forceinline__ void publish_range(int jmin, int jmax, int *range)
{
    __shared__ int smin[kWG / 64], smax[kWG / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        jmin = min(jmin, __shfl_xor(jmin, off, 64));
        jmax = max(jmax, __shfl_xor(jmax, off, 64));
    }
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        smin[w] = jmin;
        smax[w] = jmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = smin[0], b = smax[0];
        for (int q = 1; q < int(blockDim.x / 64); ++q) {
            a = min(a, smin[q]);
            b = max(b, smax[q]);
        }
        // same-address atomics serialise across the chip: only issue the ones
        // that can still move the extremes (they only ever tighten)
        if (b >= a) {
            if (a < __hip_atomic_load(range, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(range, a);
            if (b > __hip_atomic_load(range + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(range + 1, b);
        }
    }
}

template <typename T, int CHORD, bool HULL>
__global__ void __launch_bounds__(kWG) k_drop_rows(ProtonsDev p, const float *__restrict__ b,
                                                   const T *__restrict__ x, void *acc, int32_t *cnt, int *range,
                                                   const PathSrc src,  GridDev g, int64_t lo,
                                                   int64_t hi, double lambda, unsigned *status, long long *acc_lo,
                                                   const int *halt)
{
    if (gate_closed(halt)) return;
    int64_t i = lo + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    bool active = i < hi;
    Rec r{};
    double bi = 0.0;
    if (active) {
        r = load_rec(p, i);
        bi = double(b[i]);
        if (!rec_finite(r) || !isfinite(bi)) {
            raise_status(status, PCT_DEV_NONFINITE);
            active = false;
        }
    }
    DropScatterSink<T> sc;
    sc.jmin = INT_MAX;
    sc.jmax = -1;
    if (active) {
        DotSink<T> s;
        s.x = PlainX<T>{x};
        s.dot = 0.0;
        s.n2 = 0.0;
        s.re.init(r);
        {
            Merge<DotSink<T>, CHORD> m(s, g);
            walk_path<HULL>(r, src, g, m);
            m.finish();
        }
        if (s.re.unsafe) raise_status(status, PCT_DEV_REENTRY);
        if (s.n2 > 0.0) {
            sc.acc = acc;
            sc.acc_lo = acc_lo;
            sc.cnt = cnt;
            sc.status = status;
            sc.rho = lambda * (bi - s.dot) / s.n2;
            sc.re.init(r);
            Merge<DropScatterSink<T>, CHORD> m(sc, g);
            walk_path<HULL>(r, src, g, m);
            m.finish();
        }
    }
    publish_range(sc.jmin, sc.jmax, range);
}

// ---------------------------------------------------------------------------
// DROP block kernel, LPP lanes per proton.
//
// The path is monotone along its dominant in-plane axis (the lab axis closest
// to the beam direction), so a voxel can only be visited again while the path
// stays inside one slab of that axis.  The slabs the path crosses are split
// into LPP contiguous ranges, one per lane; each lane walks the pieces of the
// path inside its range.  Lanes therefore never share a voxel: merging,
// re-entry tracking, ||a_i||^2 and the once-per-row count stay lane-local, and
// the only cross-lane step is the sum of a_i.x and ||a_i||^2.
//
// Per proton: the dominant coordinate of every vertex is staged in LDS (one
// value per vertex, computed by the group's lanes in parallel); it gives the
// monotonicity check and, by binary search, each lane's first segment.  A path
// that is not monotone falls back to a single-lane walk of the whole row.
// ---------------------------------------------------------------------------
template <int LPP>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int off = LPP / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int LPP>
__device__ __forceinline__ double group_max(double v)
{
#pragma unroll
    for (int off = LPP / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

template <int LPP>
__device__ __forceinline__ bool group_any(bool p)
{
    int v = p ? 1 : 0;
#pragma unroll
    for (int off = LPP / 2; off > 0; off >>= 1) v |= __shfl_xor(v, off, 64);
    return v != 0;
}

// Per-proton path state shared by the LPP lanes of its group.  The lab
// coordinates of every vertex live in LDS (P, 3 doubles per vertex); the
// signed coordinate along the dominant axis, A(k) = sgn * P[k][dom], increases
// along a monotone path.
struct GroupPath {
    int K;           // segments of this proton's polyline
    int dom;         // dominant in-plane axis (0: x, 1: y)
    double sgn;      // direction of travel along it
    int s_lo, s_hi;  // dominant-axis index range crossed by the path (s_lo > s_hi: none)
    bool full;       // not monotone: lane 0 walks the whole row over the whole grid
};

__device__ __forceinline__ double path_A(const GroupPath &gp, const double *__restrict__ P, int k)
{
    return gp.sgn * P[3 * k + gp.dom];
}

template <int LPP, bool HULL>
__device__ __forceinline__ GroupPath stage_path(const Rec &r, const PathSrc &src, const GridDev &g,
                                                double *__restrict__ P, int l, bool active)
{
    GroupPath gp;
    gp.dom = fabs(r.cs) >= fabs(r.sn) ? 0 : 1;
    const double e = gp.dom == 0 ? r.cs : r.sn;
    gp.sgn = e > 0.0 ? 1.0 : -1.0;
    const PathState ps = path_prepare<HULL>(r, src);
    const int K = ps.nv - 1;
    gp.K = K;
    for (int k = l; k <= K; k += LPP) {
        double v[3] = {0.0, 0.0, 0.0};
        if (active) path_vertex<HULL>(r, src, ps, k, v);
        P[3 * k] = v[0];
        P[3 * k + 1] = v[1];
        P[3 * k + 2] = v[2];
    }
    __syncthreads();
    bool bad = !active;
    for (int k = l; k < K; k += LPP) bad |= !(path_A(gp, P, k + 1) > path_A(gp, P, k));
    gp.full = group_any<LPP>(bad);
    gp.s_lo = 0;
    gp.s_hi = -1;
    if (gp.full) {
        if (active) gp.s_hi = g.n[gp.dom] - 1;
        return gp;
    }
    const int a = gp.dom;
    const double c0 = P[a], c1 = P[3 * K + a];
    const double f0 = floor((fmin(c0, c1) - g.lo[a]) * g.inv_pitch[a]);
    const double f1 = floor((fmax(c0, c1) - g.lo[a]) * g.inv_pitch[a]);
    if (f1 < 0.0 || f0 > double(g.n[a] - 1)) return gp;
    gp.s_lo = int(fmax(f0, 0.0));
    gp.s_hi = int(fmin(f1, double(g.n[a] - 1)));
    return gp;
}

// The lane's share of the path: a contiguous range of dominant-axis slabs
// (lanes take consecutive ranges in the direction of travel), walked as one
// run of segments clipped to the range.  A non-monotone path is walked whole
// by lane 0.
template <int LPP, class M>
__device__ __forceinline__ void walk_lane(const GroupPath &gp, int l, const GridDev &g,
                                          const double *__restrict__ P, M &m)
{
    const int K = gp.K;
    const int a = gp.dom;
    if (gp.full) {
        if (l != 0 || gp.s_hi < gp.s_lo) return;
        for (int k = 0; k < K; ++k) {
            const double *p0 = P + 3 * k, *p1 = P + 3 * k + 3;
            m.segment(p1[0] - p0[0], p1[1] - p0[1]);
            walk_segment_range(p0, p1, g, a, 0, g.n[a] - 1, m);
        }
        return;
    }
    const int ns = gp.s_hi - gp.s_lo + 1;
    if (ns <= 0) return;
    const int q = ns / LPP, rem = ns % LPP;
    const int off = l * q + min(l, rem);
    const int cntl = q + (l < rem ? 1 : 0);
    if (cntl <= 0) return;
    int s0, s1;
    if (gp.sgn > 0.0) {
        s0 = gp.s_lo + off;
        s1 = s0 + cntl - 1;
    } else {
        s1 = gp.s_hi - off;
        s0 = s1 - cntl + 1;
    }
    // entry and exit planes of the range in signed coordinate
    const double entry = gp.sgn > 0.0 ? g.lo[a] + s0 * g.pitch[a] : -(g.lo[a] + (s1 + 1) * g.pitch[a]);
    const double exitc = gp.sgn > 0.0 ? g.lo[a] + (s1 + 1) * g.pitch[a] : -(g.lo[a] + s0 * g.pitch[a]);
    // last vertex k in [0, K-1] with A(k) <= entry
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (path_A(gp, P, mid) <= entry) lo = mid;
        else hi = mid - 1;
    }
    for (int k = lo; k < K; ++k) {
        const double *p0 = P + 3 * k, *p1 = P + 3 * k + 3;
        walk_segment_range(p0, p1, g, a, s0, s1, m);
        if (path_A(gp, P, k + 1) >= exitc) break;
    }
}

// Table-path form of the group staging: LDS holds only the signed dominant
// coordinate A(k) of every vertex (one double per vertex instead of three),
// which is all the monotonicity check and the lanes' binary searches read; a
// lane recomputes the full vertices of the segments it walks from the shared
// table, with the same arithmetic, so the walk sees the same values.
template <int LPP>
__device__ __forceinline__ GroupPath stage_path_dom(const Rec &r, const PathSrc &src, const GridDev &g,
                                                    double *__restrict__ A, int l, bool active)
{
    GroupPath gp;
    gp.dom = fabs(r.cs) >= fabs(r.sn) ? 0 : 1;
    const double e = gp.dom == 0 ? r.cs : r.sn;
    gp.sgn = e > 0.0 ? 1.0 : -1.0;
    const int K = src.K;
    gp.K = K;
    for (int k = l; k <= K; k += LPP) {
        double v[3] = {0.0, 0.0, 0.0};
        if (active) vertex(r, src.tab + k * kRowDoubles, v);
        A[k] = gp.sgn * v[gp.dom];
    }
    __syncthreads();
    bool bad = !active;
    for (int k = l; k < K; k += LPP) bad |= !(A[k + 1] > A[k]);
    gp.full = group_any<LPP>(bad);
    gp.s_lo = 0;
    gp.s_hi = -1;
    if (gp.full) {
        if (active) gp.s_hi = g.n[gp.dom] - 1;
        return gp;
    }
    const int a = gp.dom;
    const double c0 = gp.sgn * A[0], c1 = gp.sgn * A[K];  // sgn = +-1: the vertices' own coordinates
    const double f0 = floor((fmin(c0, c1) - g.lo[a]) * g.inv_pitch[a]);
    const double f1 = floor((fmax(c0, c1) - g.lo[a]) * g.inv_pitch[a]);
    if (f1 < 0.0 || f0 > double(g.n[a] - 1)) return gp;
    gp.s_lo = int(fmax(f0, 0.0));
    gp.s_hi = int(fmin(f1, double(g.n[a] - 1)));
    return gp;
}

// walk_lane over a stage_path_dom staging: the same slab range, start vertex
// and stop test, with the segment end points recomputed from the table.
template <int LPP, class M>
__device__ __forceinline__ void walk_lane_dom(const GroupPath &gp, int l, const GridDev &g,
                                              const double *__restrict__ A, const Rec &r, const PathSrc &src, M &m)
{
    const int K = gp.K;
    const int a = gp.dom;
    double p0[3], p1[3];
    if (gp.full) {
        if (l != 0 || gp.s_hi < gp.s_lo) return;
        vertex(r, src.tab, p0);
        for (int k = 0; k < K; ++k) {
            vertex(r, src.tab + (k + 1) * kRowDoubles, p1);
            m.segment(p1[0] - p0[0], p1[1] - p0[1]);
            walk_segment_range(p0, p1, g, a, 0, g.n[a] - 1, m);
            p0[0] = p1[0];
            p0[1] = p1[1];
            p0[2] = p1[2];
        }
        return;
    }
    const int ns = gp.s_hi - gp.s_lo + 1;
    if (ns <= 0) return;
    const int q = ns / LPP, rem = ns % LPP;
    const int off = l * q + min(l, rem);
    const int cntl = q + (l < rem ? 1 : 0);
    if (cntl <= 0) return;
    int s0, s1;
    if (gp.sgn > 0.0) {
        s0 = gp.s_lo + off;
        s1 = s0 + cntl - 1;
    } else {
        s1 = gp.s_hi - off;
        s0 = s1 - cntl + 1;
    }
    const double entry = gp.sgn > 0.0 ? g.lo[a] + s0 * g.pitch[a] : -(g.lo[a] + (s1 + 1) * g.pitch[a]);
    const double exitc = gp.sgn > 0.0 ? g.lo[a] + (s1 + 1) * g.pitch[a] : -(g.lo[a] + s0 * g.pitch[a]);
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A[mid] <= entry) lo = mid;
        else hi = mid - 1;
    }
    vertex(r, src.tab + lo * kRowDoubles, p0);
    for (int k = lo; k < K; ++k) {
        vertex(r, src.tab + (k + 1) * kRowDoubles, p1);
        walk_segment_range(p0, p1, g, a, s0, s1, m);
        if (A[k + 1] >= exitc) break;
        p0[0] = p1[0];
        p0[1] = p1[1];
        p0[2] = p1[2];
    }
}

// Staging and lane walk of the binned and separate-commit block kernels: hull
// paths keep every vertex in LDS (a hull vertex costs two quadratures), table
// paths only A(k).
template <int LPP, bool HULL>
__device__ __forceinline__ GroupPath stage_group(const Rec &r, const PathSrc &src, const GridDev &g, double *P,
                                                 int l, bool active)
{
    if constexpr (HULL)
        return stage_path<LPP, true>(r, src, g, P, l, active);
    else
        return stage_path_dom<LPP>(r, src, g, P, l, active);
}

template <int LPP, bool HULL, class M>
__device__ __forceinline__ void walk_group_lane(const GroupPath &gp, int l, const GridDev &g, const double *P,
                                                const Rec &r, const PathSrc &src, M &m)
{
    if constexpr (HULL)
        walk_lane<LPP>(gp, l, g, P, m);
    else
        walk_lane_dom<LPP>(gp, l, g, P, r, src, m);
}

// Doubles of LDS a group's staging takes per vertex.
template <bool HULL>
constexpr int kStageDoubles = HULL ? 3 : 1;

// Walk sink of the block kernel: tracks re-entries, accumulates ||a_i||^2 and
// stashes the lane's merged pieces (voxel | first-visit bit, chord) in LDS,
// entry-major so that the lanes of a wave hit different banks.
template <typename CT, int S>
struct StashSink {
    int *__restrict__ sj;
    CT *__restrict__ sc;
    int lane;
    Reentry re;
    double n2;
    int count;
    __device__ __forceinline__ void segment(double dx, double dy) { re.segment(dx, dy); }
    __device__ __forceinline__ void final(int j, int ix, int iy, int iz, double c)
    {
        bool first;
        const double aprev = re.visit(j, ix, iy, iz, c, first);
        n2 += c * (2.0 * aprev + c);
        if (count < S) {
            sj[count * 64 + lane] = first ? (j | int(0x80000000u)) : j;
            sc[count * 64 + lane] = CT(c);
        }
        ++count;
    }
};

constexpr int kStash = 12;  // pieces per lane kept in LDS; longer lanes walk again

template <typename T>
__host__ __device__ constexpr size_t stash_bytes()
{
    return size_t(64) * kStash * (sizeof(int) + (sizeof(T) == 4 ? sizeof(float) : sizeof(double)));
}

// Fused DROP block kernel: one wave per workgroup, 64 / LPP protons per wave.
template <typename T, int CHORD, int LPP, bool HULL>
__global__ void __launch_bounds__(64) k_drop_block(ProtonsDev p, const float *__restrict__ b,
                                                   const T *__restrict__ x, void *acc, int32_t *cnt, int *range,
                                                   const PathSrc src,  GridDev g, int64_t lo,
                                                   int64_t hi, double lambda, unsigned *status, long long *acc_lo,
                                                   const int *halt)
{
    if (gate_closed(halt)) return;
    using CT = typename std::conditional<sizeof(T) == 4, float, double>::type;
    extern __shared__ double lds[];
    constexpr int GPW = 64 / LPP;  // proton groups per workgroup
    const int lane = threadIdx.x;
    const int grp = lane / LPP;
    const int l = lane % LPP;
    const int64_t i = lo + int64_t(blockIdx.x) * GPW + grp;
    bool active = i < hi;
    Rec r{};
    double bi = 0.0;
    if (active) {
        r = load_rec(p, i);
        bi = double(b[i]);
        if (!rec_finite(r) || !isfinite(bi)) {
            if (l == 0) raise_status(status, PCT_DEV_NONFINITE);
            active = false;
        }
    }
    if (!active) r.cs = 1.0, r.sn = 0.0;
    double *P = lds + grp * kStageDoubles<HULL> * src.nvmax;
    char *stash = reinterpret_cast<char *>(lds + GPW * kStageDoubles<HULL> * src.nvmax);
    int *sj = reinterpret_cast<int *>(stash);
    CT *sc = reinterpret_cast<CT *>(stash + size_t(64) * kStash * sizeof(int));
    const GroupPath gp = stage_group<LPP, HULL>(r, src, g, P, l, active);

    // one walk: ||a_i||^2, re-entries and the stash of pieces
    StashSink<CT, kStash> st{sj, sc, lane, {}, 0.0, 0};
    st.re.init(r);
    {
        Merge<StashSink<CT, kStash>, CHORD> m(st, g);
        walk_group_lane<LPP, HULL>(gp, l, g, P, r, src, m);
        m.finish();
    }
    if (st.re.unsafe) raise_status(status, PCT_DEV_REENTRY);
    const bool spill = st.count > kStash;
    const int ns = min(st.count, kStash);
    // a_i . x: gathers from the stash (independent loads)
    double dot = 0.0;
    if (!spill) {
#pragma unroll 4
        for (int q = 0; q < ns; ++q) {
            const int j = sj[q * 64 + lane] & 0x7FFFFFFF;
            dot += double(sc[q * 64 + lane]) * double(x[j]);
        }
    } else {
        DotSink<T> ds;
        ds.x = PlainX<T>{x};
        ds.dot = 0.0;
        ds.n2 = 0.0;
        ds.re.init(r);
        Merge<DotSink<T>, CHORD> m(ds, g);
        walk_group_lane<LPP, HULL>(gp, l, g, P, r, src, m);
        m.finish();
        dot = ds.dot;
    }
    dot = group_sum<LPP>(dot);
    const double n2 = group_sum<LPP>(st.n2);
    int jmin = INT_MAX, jmax = -1;
    if (n2 > 0.0) {
        const double rho = lambda * (bi - dot) / n2;
        if (!spill) {
            for (int q = 0; q < ns; ++q) {
                const int e = sj[q * 64 + lane];
                const int j = e & 0x7FFFFFFF;
                const bool first = e < 0;
                const double v = rho * double(sc[q * 64 + lane]);
                scatter_one<T>(acc, acc_lo, cnt, j, v, first, status);
                jmin = min(jmin, j);
                jmax = max(jmax, j);
            }
        } else {
            DropScatterSink<T> sc2;
            sc2.acc = acc;
            sc2.acc_lo = acc_lo;
            sc2.cnt = cnt;
            sc2.status = status;
            sc2.rho = rho;
            sc2.jmin = INT_MAX;
            sc2.jmax = -1;
            sc2.re.init(r);
            Merge<DropScatterSink<T>, CHORD> m(sc2, g);
            walk_group_lane<LPP, HULL>(gp, l, g, P, r, src, m);
            m.finish();
            jmin = sc2.jmin;
            jmax = sc2.jmax;
        }
    }
    publish_range(jmin, jmax, range);
}

// ---------------------------------------------------------------------------
// Fused FP32 DROP sweep: the commit of block q-1 happens inside the launch of
// block q.
//
// Two copies of the iterate (X0 = the caller's x, X1 in the workspace) and
// three packed accumulators rotate with the block index q of the sweep:
//   base = X[q % 2] holds every block before q-1;  PK[(q-1) % 3] holds block
//   q-1's sums.  Block q reads  xbar_j = base_j + sum_j / s_j  (the committed
//   value of block q-1, computed on the fly) and scatters into PK[q % 3].
//   In the same launch, commit workgroups write X[(q+1) % 2] = base + update
//   over the index ranges of blocks q-1 and q-2 (the only places where the two
//   copies differ) and clear PK[(q-2) % 3].  Nothing read in a launch is
//   written in it, so no grid-wide synchronisation is needed, and the commit's
//   memory traffic overlaps the walk.  A flush kernel ends the sweep.
// Range slots rotate over 4: block q accumulates slot q%4, reads q-1 and q-2,
// and re-arms slot (q+1)%4 for the next block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float committed_value(float base, unsigned long long w)
{
    if (w == 0ull) return base;
    int c;
    double sum;
    unpack_accumulator(w, c, sum);
    return float(double(base) + sum / double(c));
}

struct LazyX {
    const float *__restrict__ base;
    const unsigned long long *__restrict__ pk;
    __device__ __forceinline__ double operator()(int j) const { return double(committed_value(base[j], pk[j])); }
};

__device__ __forceinline__ void commit_part(const float *__restrict__ base, float *__restrict__ next,
                                            const unsigned long long *__restrict__ pk_prev,
                                            unsigned long long *__restrict__ pk_old, const int *r_prev,
                                            const int *r_old, int *r_reset, int nvox, int wg, int n_wg,
                                            int full = 0)
{
    // full: the whole volume instead of the published ranges
    const int j0 = full ? 0 : min(r_prev[0], r_old[0]);
    const int j1 = full ? nvox - 1 : max(r_prev[1], r_old[1]);
    if (wg == 0 && threadIdx.x == 0) {
        r_reset[0] = INT_MAX;
        r_reset[1] = -1;
    }
    if (j1 < j0 || j0 < 0) return;
    const int stride = 4 * n_wg * int(blockDim.x);
    for (int j = (j0 & ~3) + 4 * (wg * int(blockDim.x) + int(threadIdx.x)); j <= j1; j += stride) {
        const ulonglong2 p01 = *reinterpret_cast<const ulonglong2 *>(pk_prev + j);
        const ulonglong2 p23 = *reinterpret_cast<const ulonglong2 *>(pk_prev + j + 2);
        const ulonglong2 o01 = *reinterpret_cast<const ulonglong2 *>(pk_old + j);
        const ulonglong2 o23 = *reinterpret_cast<const ulonglong2 *>(pk_old + j + 2);
        const unsigned long long wp[4] = {p01.x, p01.y, p23.x, p23.y};
        const unsigned long long wo[4] = {o01.x, o01.y, o23.x, o23.y};
        // next differs from base only where block q-1 or q-2 touched a voxel
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int jj = j + e;
            if ((wp[e] | wo[e]) != 0ull && jj < nvox) next[jj] = committed_value(base[jj], wp[e]);
            if (wo[e] != 0ull) pk_old[jj] = 0ull;
        }
    }
}

constexpr int kCommitWG = 1024;  // commit workgroups (64 threads) per fused launch
static_assert(kCommitWG % 8 == 0, "proton workgroups must start on XCD 0");

// Four waves per SIMD (at most 128 VGPRs): the walk is latency-bound, and the
// extra wave hides more latency than the few spilled registers cost.
template <int CHORD, int LPP, bool HULL>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) k_drop_fused(ProtonsDev p, const float *__restrict__ b,
                                                   const float *__restrict__ base, float *__restrict__ next,
                                                   const unsigned long long *__restrict__ pk_prev,
                                                   unsigned long long *pk_cur, unsigned long long *pk_old, int *r_cur,
                                                   const int *r_prev, const int *r_old, int *r_reset,
                                                   const PathSrc src,  GridDev g, int64_t lo,
                                                   int64_t hi, double lambda, unsigned *status, int nvox,
                                                   int full)
{
    if (int(blockIdx.x) < kCommitWG) {
        commit_part(base, next, pk_prev, pk_old, r_prev, r_old, r_reset, nvox, int(blockIdx.x), kCommitWG, full);
        return;
    }
    using CT = float;
    extern __shared__ double lds[];
    constexpr int GPW = 64 / LPP;
    const int lane = threadIdx.x;
    const int grp = lane / LPP;
    const int l = lane % LPP;
    // XCD-aware placement: workgroup w runs on XCD w mod 8, so the proton
    // workgroups are dealt to the eight XCDs in contiguous runs of the block
    // (8 * per_xcd workgroups are launched; the padding ones idle).  With the
    // block ordered by entry slice and lateral position, each XCD then walks
    // a band of neighbouring paths and finds their voxels in its own L2.
    const int wq = int(blockIdx.x) - kCommitWG;
    const int64_t n_wg = (hi - lo + GPW - 1) / GPW;
    const int64_t per_xcd = (n_wg + 7) / 8;
    const int64_t wg = int64_t(wq % 8) * per_xcd + wq / 8;
    const int64_t i = lo + wg * GPW + grp;
    bool active = wg < n_wg && i < hi;
    Rec r{};
    double bi = 0.0;
    if (active) {
        r = load_rec(p, i);
        bi = double(b[i]);
        if (!rec_finite(r) || !isfinite(bi)) {
            if (l == 0) raise_status(status, PCT_DEV_NONFINITE);
            active = false;
        }
    }
    if (!active) r.cs = 1.0, r.sn = 0.0;
    double *P = lds + grp * 3 * src.nvmax;
    char *stash = reinterpret_cast<char *>(lds + GPW * 3 * src.nvmax);
    int *sj = reinterpret_cast<int *>(stash);
    CT *sc = reinterpret_cast<CT *>(stash + size_t(64) * kStash * sizeof(int));
    const GroupPath gp = stage_path<LPP, HULL>(r, src, g, P, l, active);

    StashSink<CT, kStash> st{sj, sc, lane, {}, 0.0, 0};
    st.re.init(r);
    {
        Merge<StashSink<CT, kStash>, CHORD> m(st, g);
        walk_lane<LPP>(gp, l, g, P, m);
        m.finish();
    }
    if (st.re.unsafe) raise_status(status, PCT_DEV_REENTRY);
    const bool spill = st.count > kStash;
    const int ns = min(st.count, kStash);
    const LazyX xa{base, pk_prev};
    double dot = 0.0;
    if (!spill) {
#pragma unroll 4
        for (int q = 0; q < ns; ++q) {
            const int j = sj[q * 64 + lane] & 0x7FFFFFFF;
            dot += double(sc[q * 64 + lane]) * xa(j);
        }
    } else {
        DotSink<float, LazyX> ds;
        ds.x = xa;
        ds.dot = 0.0;
        ds.n2 = 0.0;
        ds.re.init(r);
        Merge<DotSink<float, LazyX>, CHORD> m(ds, g);
        walk_lane<LPP>(gp, l, g, P, m);
        m.finish();
        dot = ds.dot;
    }
    dot = group_sum<LPP>(dot);
    const double n2 = group_sum<LPP>(st.n2);
    int jmin = INT_MAX, jmax = -1;
    if (n2 > 0.0) {
        const double rho = lambda * (bi - dot) / n2;
        if (!spill) {
            for (int q = 0; q < ns; ++q) {
                const int e = sj[q * 64 + lane];
                const int j = e & 0x7FFFFFFF;
                atomicAdd(pk_cur + j, pack_contribution(rho * double(sc[q * 64 + lane]), e < 0, status));
                jmin = min(jmin, j);
                jmax = max(jmax, j);
            }
        } else {
            DropScatterSink<float> sc2;
            sc2.acc = pk_cur;
            sc2.cnt = nullptr;
            sc2.status = status;
            sc2.rho = rho;
            sc2.jmin = INT_MAX;
            sc2.jmax = -1;
            sc2.re.init(r);
            Merge<DropScatterSink<float>, CHORD> m(sc2, g);
            walk_lane<LPP>(gp, l, g, P, m);
            m.finish();
            jmin = sc2.jmin;
            jmax = sc2.jmax;
        }
    }
    if (!full) publish_range(jmin, jmax, r_cur);   // full is uniform over the launch
}

// ---------------------------------------------------------------------------
// Traced-ahead schedule (FP32, 64 lanes per proton).  The rows do not depend
// on x, so launch q traces the rows of block q+1 while it runs the DROP
// update of block q from the rows traced in launch q-1 (and commits block
// q-1 as in k_drop_fused): the walk leaves the chain of dependent block
// steps.  A row record holds the image of the lane stash (kStash entries x
// 64 lanes, entry-major), the lane piece counts and ||a_i||^2; a lane whose
// count exceeds kStash walks its slabs again in the DROP step, exactly as in
// k_drop_fused, so both schedules give bitwise the same result.
// ---------------------------------------------------------------------------
struct SlotDev {
    int *vox;      // [record][kStash][64]
    float *chord;  // [record][kStash][64]
    int *cnt;      // [record][64]
    double *n2;    // [record]
};

static_assert(kSlotRecordBytes == size_t(kStash) * 64 * (sizeof(int) + sizeof(float)) + 64 * sizeof(int) +
                                      sizeof(double),
              "row record layout");

__host__ __device__ inline SlotDev slot_at(char *base, int64_t records)
{
    SlotDev d;
    d.vox = reinterpret_cast<int *>(base);
    d.chord = reinterpret_cast<float *>(base + size_t(records) * kStash * 64 * sizeof(int));
    d.cnt = reinterpret_cast<int *>(base + size_t(records) * kStash * 64 * (sizeof(int) + sizeof(float)));
    d.n2 = reinterpret_cast<double *>(base + size_t(records) * (kStash * 64 * (sizeof(int) + sizeof(float)) +
                                                                64 * sizeof(int)));
    return d;
}

// Trace of record r of the block [wlo, whi) into slot wr (one proton per
// one-wave workgroup).
template <int CHORD, bool HULL>
__device__ __forceinline__ void trace_role(const ProtonsDev &p, const SlotDev &wr, const PathSrc src,
                                            const GridDev &g, int64_t wlo, int64_t whi, int64_t r, double *P,
                                           int *sj, float *sc, unsigned *status)
{
    const int lane = threadIdx.x;
    const int64_t i = wlo + r;
    if (i >= whi) return;  // uniform: one proton per workgroup
    Rec rec = load_rec(p, i);
    bool active = true;
    if (!rec_finite(rec)) {
        if (lane == 0) raise_status(status, PCT_DEV_NONFINITE);
        active = false;
        rec.cs = 1.0;
        rec.sn = 0.0;
    }
    const GroupPath gp = stage_path<64, HULL>(rec, src, g, P, lane, active);
    StashSink<float, kStash> st{sj, sc, lane, {}, 0.0, 0};
    st.re.init(rec);
    {
        Merge<StashSink<float, kStash>, CHORD> m(st, g);
        walk_lane<64>(gp, lane, g, P, m);
        m.finish();
    }
    if (st.re.unsafe) raise_status(status, PCT_DEV_REENTRY);
    const double n2 = group_sum<64>(st.n2);
    const int ns = min(st.count, kStash);
    for (int k = 0; k < ns; ++k) {
        const int64_t q = (r * kStash + k) * 64 + lane;
        wr.vox[q] = sj[k * 64 + lane];
        wr.chord[q] = sc[k * 64 + lane];
    }
    wr.cnt[r * 64 + lane] = active ? st.count : 0;
    if (lane == 0) wr.n2[r] = active ? n2 : 0.0;
}

template <int CHORD, bool HULL>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_drop_pipe(ProtonsDev p, const float *__restrict__ b, const float *__restrict__ base, float *__restrict__ next,
            const unsigned long long *__restrict__ pk_prev, unsigned long long *pk_cur, unsigned long long *pk_old,
            int *r_cur, const int *r_prev, const int *r_old, int *r_reset, SlotDev rd, SlotDev wr,
            const PathSrc src,  GridDev g, int64_t lo, int64_t hi, int64_t wlo, int64_t whi,
            int n_commit, double lambda, unsigned *status, int nvox, int full)
{
    const int bid = int(blockIdx.x);
    if (bid < n_commit) {
        commit_part(base, next, pk_prev, pk_old, r_prev, r_old, r_reset, nvox, bid, n_commit, full);
        return;
    }
    extern __shared__ double lds[];
    double *P = lds;
    char *stash = reinterpret_cast<char *>(lds + 3 * src.nvmax);
    int *sj = reinterpret_cast<int *>(stash);
    float *sc = reinterpret_cast<float *>(stash + size_t(64) * kStash * sizeof(int));
    const int lane = threadIdx.x;
    // workgroups: [commit | trace of block q+1 | DROP step of block q]; the
    // trace, the longer chain, is dispatched first
    const int64_t n_d = hi - lo;
    const int64_t per_xcd = (n_d + 7) / 8;
    const int64_t n_w8 = 8 * ((whi - wlo + 7) / 8);  // keeps the DROP workgroups XCD-aligned
    if (bid - n_commit < n_w8) {
        trace_role<CHORD, HULL>(p, wr, src, g, wlo, whi, int64_t(bid - n_commit), P, sj, sc, status);
        return;
    }
    const int wq = int(bid - n_commit - n_w8);
    {
        // ---- DROP step of block q from its traced rows (XCD-aware placement)
        const int64_t r = int64_t(wq % 8) * per_xcd + wq / 8;
        bool active = r < n_d;
        const int64_t i = lo + r;
        double bi = 0.0, n2 = 0.0;
        int cnt = 0;
        if (active) {
            bi = double(b[i]);
            n2 = rd.n2[r];
            cnt = rd.cnt[r * 64 + lane];
            if (!isfinite(bi)) {
                if (lane == 0) raise_status(status, PCT_DEV_NONFINITE);
                active = false;
            }
        }
        const bool spill = cnt > kStash;
        const bool any_spill = group_any<64>(spill);
        const LazyX xa{base, pk_prev};
        int jr[kStash];
        float cr[kStash];
        double dot = 0.0;
#pragma unroll
        for (int k = 0; k < kStash; ++k) {
            jr[k] = 0;
            cr[k] = 0.f;
            if (!spill && k < cnt) {
                const int64_t q = (r * kStash + k) * 64 + lane;
                jr[k] = rd.vox[q];
                cr[k] = rd.chord[q];
            }
        }
#pragma unroll
        for (int k = 0; k < kStash; ++k)
            if (!spill && k < cnt) dot += double(cr[k]) * xa(jr[k] & 0x7FFFFFFF);
        Rec rec{};
        GroupPath gp{};
        if (any_spill) {
            // lanes beyond the stash walk their slabs again (rare)
            if (active) rec = load_rec(p, i);
            if (!active) rec.cs = 1.0, rec.sn = 0.0;
            gp = stage_path<64, HULL>(rec, src, g, P, lane, active);
            if (spill) {
                DotSink<float, LazyX> ds;
                ds.x = xa;
                ds.dot = 0.0;
                ds.n2 = 0.0;
                ds.re.init(rec);
                Merge<DotSink<float, LazyX>, CHORD> m(ds, g);
                walk_lane<64>(gp, lane, g, P, m);
                m.finish();
                dot = ds.dot;
            }
        }
        dot = group_sum<64>(dot);
        int jmin = INT_MAX, jmax = -1;
        if (active && n2 > 0.0) {
            const double rho = lambda * (bi - dot) / n2;
            if (!spill) {
#pragma unroll
                for (int k = 0; k < kStash; ++k) {
                    if (k < cnt) {
                        const int e = jr[k];
                        const int j = e & 0x7FFFFFFF;
                        atomicAdd(pk_cur + j, pack_contribution(rho * double(cr[k]), e < 0, status));
                        jmin = min(jmin, j);
                        jmax = max(jmax, j);
                    }
                }
            } else {
                DropScatterSink<float> sc2;
                sc2.acc = pk_cur;
                sc2.cnt = nullptr;
                sc2.status = status;
                sc2.rho = rho;
                sc2.jmin = INT_MAX;
                sc2.jmax = -1;
                sc2.re.init(rec);
                Merge<DropScatterSink<float>, CHORD> m(sc2, g);
                walk_lane<64>(gp, lane, g, P, m);
                m.finish();
                jmin = sc2.jmin;
                jmax = sc2.jmax;
            }
        }
        if (!full) publish_range(jmin, jmax, r_cur);   // full is uniform over the launch
    }
}

// Start of a fused sweep: X1 = x, all range slots empty.
__global__ void __launch_bounds__(256) k_sweep_begin(const float *__restrict__ x, float *__restrict__ x1, int *slots,
                                                     int nvox)
{
    const int t = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (t < 8 && blockIdx.x == 0) slots[t] = (t & 1) ? -1 : INT_MAX;
    for (int j = t; j < nvox; j += int(gridDim.x * blockDim.x)) x1[j] = x[j];
}

// End of a fused sweep of T blocks: x = X[T%2] + update of block T-1 over the
// ranges of blocks T-1 and T-2; clears the accumulators of both.
__global__ void __launch_bounds__(256) k_sweep_end(float *x, const float *src, unsigned long long *pk_last,
                                                   unsigned long long *pk_prev, const int *r_last, const int *r_prev,
                                                   int nvox, int full)
{
    // full: the whole volume instead of the published ranges
    const int j0 = full ? 0 : min(r_last[0], r_prev[0]);
    const int j1 = full ? nvox - 1 : max(r_last[1], r_prev[1]);
    if (j1 < j0 || j0 < 0) return;
    for (int j = j0 + int(blockIdx.x * blockDim.x + threadIdx.x); j <= j1 && j < nvox;
         j += int(gridDim.x * blockDim.x)) {
        const unsigned long long w = pk_last[j];
        x[j] = committed_value(src[j], w);
        if (w != 0ull) pk_last[j] = 0ull;
        if (pk_prev[j] != 0ull) pk_prev[j] = 0ull;
    }
}

// ---------------------------------------------------------------------------
// Binned FP32 schedule: the block's D-weighted back-projection is staged per
// slab of the block's dominant axis and summed in LDS, one workgroup per slab.
//
// Launch 1 (k_drop_bin) runs the proton groups exactly as k_drop_fused does
// (walk, a_i.x against the committed iterate, ||a_i||^2, rho_i), but each lane
// stores its packed contributions (the same 64-bit word: row count bit plus
// rho_i a_ij in fixed point) into the bin of the piece's slab,
// bins[s][p][0..kBinCap), with the number of entries in cnt[s][p].  Lanes own
// disjoint slab ranges, so every (slab, proton) bin has a single writer: plain
// stores, no atomics.  Pieces without a bin (a proton whose dominant axis is
// not the block's, a path that is not monotone along it, more than kBinCap
// pieces of one row in one slab) go to a packed overflow accumulator with a
// global atomic, and raise the block's overflow flag.
//
// Launch 2 (k_slab_commit) gives each slab (and z chunk) of the block's axis
// to one workgroup: it adds the slab's bin entries into a dense LDS window of
// the slab (64-bit integer adds), adds the overflow words of the window when
// the flag is up, and commits x_j = x_j + sum_j / s_j for every voxel of the
// window the block touched.  The integer sums per voxel are the ones the
// atomic schedules form, so without compensation the result is bitwise
// theirs; slabs are disjoint, so the commit is a plain read-modify-write of x
// over exactly the touched voxels.
//
// Compensation (default): the commit keeps the rounding error of the FP32
// iterate in a second FP32 word per voxel (lo, zero at the start of a call),
// forms base = x_j + lo_j + sum_j / s_j in FP64 and stores x_j = fl32(base),
// lo_j = fl32(base - x_j).  The gathers read x_j (the FP32 high part); x_j is
// the iterate rounded once, whatever the number of commits.
// ---------------------------------------------------------------------------
constexpr int kSlabWG = 1024;  // threads of a slab-commit workgroup

struct BinsDev {
    unsigned long long *w;  // [slab][kBinCap][cap]: packed words, entry-major (a slab's first
                            // entries are contiguous)
    unsigned *j1;           // [slab][kBinCap - 1][cap]: voxel index of entries 1.. of each bin
    unsigned *j0;           // [parity][slab][cap]: voxel index of entry 0 | (entries - 1) << 30,
                            // kEmptyBin for a bin without entries
    float *rowmax;          // [cap]: largest |rho_i a_ij| of each row of the block
    int cap;                // rows per block the bins hold (a multiple of 16)
    int nslab;              // max(nx, ny)
};
constexpr unsigned kEmptyBin = 0xFFFFFFFFu;

// Dominant in-plane axis of the block, from its first record's gantry angle.
// It only routes pieces (rows of the other axis go to the overflow words,
// whose integer sums are the same), so a single-precision hardware cosine
// serves, the same in every kernel of the block.
__device__ __forceinline__ int block_axis(const ProtonsDev &p, int64_t lo)
{
    const float c = __cosf(p.gantry[lo]);
    return c * c >= 0.5f ? 0 : 1;
}

// Exact quotient floor(j / d) for j < 2^31 and 1 <= d < 2^30, from an FP64
// product with inv = 1 / d: the product is within 2^-20 of j / d, so the
// truncated quotient is off by at most one and one remainder test corrects
// it (a handful of instructions instead of the integer division sequence).
__device__ __forceinline__ unsigned udiv_exact(unsigned j, unsigned d, double inv)
{
    unsigned q = unsigned(double(j) * inv);
    const int r = int(j - q * d);
    if (r < 0) --q;
    else if (r >= int(d)) ++q;
    return q;
}

// One lane's pieces, in walk order (slab by slab in the direction of travel),
// into the bins of row p of the block.  A slab's first entry is held until the
// lane leaves the slab, then stored with the bin's entry count in the top bits
// of its voxel word; further entries are stored as they come.
struct BinWriter {
    BinsDev bins;
    int par, axis, nx, ny;
    int p;
    bool direct;  // the row has no bins: every piece to the overflow accumulator
    unsigned long long *ovf;
    int *ovf_flag;
    int cur, k;
    unsigned long long w0;
    unsigned j0;
    double inv_nx, inv_ny;  // 1 / nx, 1 / ny

    __device__ __forceinline__ void overflow(unsigned j, unsigned long long w)
    {
        atomicAdd(ovf + j, w);
        *ovf_flag = 1;
    }
    __device__ __forceinline__ void flush()
    {
        if (cur >= 0) {
            const size_t q = size_t(cur) * bins.cap + p;
            bins.w[size_t(cur) * kBinCap * bins.cap + p] = w0;
            bins.j0[size_t(par) * bins.nslab * bins.cap + q] = j0 | (unsigned(min(k, kBinCap) - 1) << 30);
        }
        cur = -1;
    }
    __device__ __forceinline__ void put(int jj, unsigned long long w)
    {
        const unsigned j = unsigned(jj);
        if (direct) {
            overflow(j, w);
            return;
        }
        const unsigned row = udiv_exact(j, unsigned(nx), inv_nx);  // j / nx
        const int s = axis == 0 ? int(j - row * unsigned(nx))
                                : int(row - udiv_exact(row, unsigned(ny), inv_ny) * unsigned(ny));
        if (s != cur) {
            flush();
            cur = s;
            k = 0;
        }
        if (k == 0) {
            w0 = w;
            j0 = j;
        } else if (k < kBinCap) {
            bins.w[(size_t(s) * kBinCap + k) * bins.cap + p] = w;
            bins.j1[(size_t(s) * (kBinCap - 1) + (k - 1)) * bins.cap + p] = j;
        } else {
            overflow(j, w);
        }
        ++k;
    }
};

// Walk sink of a lane that re-walks its slabs (stash overflow): packed
// contributions straight into the bins.
struct BinScatterSink {
    BinWriter *bw;
    unsigned *status;
    Reentry re;
    double rho;
    double cmax;  // largest |rho a_ij| of the lane's pieces
    __device__ __forceinline__ void segment(double dx, double dy) { re.segment(dx, dy); }
    __device__ __forceinline__ void final(int j, int ix, int iy, int iz, double c)
    {
        bool first;
        re.visit(j, ix, iy, iz, c, first);
        const double v = rho * c;
        cmax = fmax(cmax, fabs(v));
        bw->put(j, pack_contribution(v, first, status));
    }
};

template <int CHORD, int LPP, bool HULL>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_drop_bin(ProtonsDev p, const float *__restrict__ b, const float *__restrict__ x, BinsDev bins, int par,
           unsigned long long *ovf, int *ovf_flag, const PathSrc src, GridDev g, int64_t lo, int64_t hi,
           double lambda, unsigned *status, const int *halt)
{
    if (gate_closed(halt)) return;
    // also writes bins.rowmax[i - lo]: the row's largest |rho_i a_ij| (0 for a skipped row)
    using CT = float;
    extern __shared__ double lds[];
    constexpr int GPW = 64 / LPP;
    const int lane = threadIdx.x;
    const int grp = lane / LPP;
    const int l = lane % LPP;
    // XCD-aware placement as in k_drop_fused: contiguous runs of the block per XCD
    const int wq = int(blockIdx.x);
    const int64_t n_wg = (hi - lo + GPW - 1) / GPW;
    const int64_t per_xcd = (n_wg + 7) / 8;
    const int64_t wg = int64_t(wq % 8) * per_xcd + wq / 8;
    const int64_t i = lo + wg * GPW + grp;
    bool active = wg < n_wg && i < hi;
    Rec r{};
    double bi = 0.0;
    if (active) {
        r = load_rec(p, i);
        bi = double(b[i]);
        if (!rec_finite(r) || !isfinite(bi)) {
            if (l == 0) raise_status(status, PCT_DEV_NONFINITE);
            active = false;
        }
    }
    if (!active) r.cs = 1.0, r.sn = 0.0;
    double *P = lds + grp * kStageDoubles<HULL> * src.nvmax;
    char *stash = reinterpret_cast<char *>(lds + GPW * kStageDoubles<HULL> * src.nvmax);
    int *sj = reinterpret_cast<int *>(stash);
    CT *sc = reinterpret_cast<CT *>(stash + size_t(64) * kStash * sizeof(int));
    const GroupPath gp = stage_group<LPP, HULL>(r, src, g, P, l, active);

    StashSink<CT, kStash> st{sj, sc, lane, {}, 0.0, 0};
    st.re.init(r);
    {
        Merge<StashSink<CT, kStash>, CHORD> m(st, g);
        walk_group_lane<LPP, HULL>(gp, l, g, P, r, src, m);
        m.finish();
    }
    if (st.re.unsafe) raise_status(status, PCT_DEV_REENTRY);
    const bool spill = st.count > kStash;
    const int ns = min(st.count, kStash);
    const PlainX<float> xa{x};
    double dot = 0.0;
    if (!spill) {
#pragma unroll 4
        for (int q = 0; q < ns; ++q) {
            const int j = sj[q * 64 + lane] & 0x7FFFFFFF;
            dot += double(sc[q * 64 + lane]) * xa(j);
        }
    } else {
        DotSink<float> ds;
        ds.x = xa;
        ds.dot = 0.0;
        ds.n2 = 0.0;
        ds.re.init(r);
        Merge<DotSink<float>, CHORD> m(ds, g);
        walk_group_lane<LPP, HULL>(gp, l, g, P, r, src, m);
        m.finish();
        dot = ds.dot;
    }
    dot = group_sum<LPP>(dot);
    const double n2 = group_sum<LPP>(st.n2);
    double cmax = 0.0;
    if (n2 > 0.0) {
        const double rho = lambda * (bi - dot) / n2;
        const int axis = block_axis(p, lo);
        BinWriter bw{bins,     par, axis, g.n[0], g.n[1], int(i - lo), gp.full || gp.dom != axis, ovf, ovf_flag, -1,
                     0,        0ull, 0u,  g.inv_n[0], g.inv_n[1]};
        if (!spill) {
            for (int q = 0; q < ns; ++q) {
                const int e = sj[q * 64 + lane];
                const double v = rho * double(sc[q * 64 + lane]);
                cmax = fmax(cmax, fabs(v));
                bw.put(e & 0x7FFFFFFF, pack_contribution(v, e < 0, status));
            }
        } else {
            BinScatterSink ss{&bw, status, {}, rho, 0.0};
            ss.re.init(r);
            Merge<BinScatterSink, CHORD> m(ss, g);
            walk_group_lane<LPP, HULL>(gp, l, g, P, r, src, m);
            m.finish();
            cmax = ss.cmax;
        }
        bw.flush();
    }
    cmax = group_max<LPP>(cmax);
    if (l == 0 && wg < n_wg && i < hi) bins.rowmax[i - lo] = float(cmax);
}

// Start of a binned sweep: every bin of both parities empty and both overflow
// flags zero.
__global__ void __launch_bounds__(256) k_bins_begin(unsigned *j0, size_t n, int *ovf_flag)
{
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < 2) ovf_flag[t] = 0;
    uint4 *c4 = reinterpret_cast<uint4 *>(j0);
    for (size_t q = t; q < n / 4; q += size_t(gridDim.x) * blockDim.x)
        c4[q] = make_uint4(kEmptyBin, kEmptyBin, kEmptyBin, kEmptyBin);
}

__global__ void __launch_bounds__(256) k_zero_f32(float *v, int64_t n)
{
    for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += int64_t(gridDim.x) * blockDim.x)
        v[q] = 0.f;
}

// Commit of block [lo, lo + nb) of the binned schedule: workgroup
// (slab s, z chunk zi) sums the slab's bins into its LDS window and commits
// the touched voxels.  Workgroups of chunk 0 also empty the other parity's
// bins of their slab (read by the previous block's commit) and clear the other
// parity's overflow flag.  Thread t takes rows t, t + kSlabWG, ... of the
// block: the first entries of its rows are read coalesced, all at once, then
// the second entries of the rows that have them, then the rare rest; in the
// commit it takes a fixed set of window cells whose x loads are issued before
// any store.
constexpr int kRowsPerThread = 8;   // rows of a block per slab-commit thread
constexpr int kCommitCells = 16;    // window cells per thread and pass of the commit

// Window cell of voxel j in the slab's z range [z0, z1), or -1.
// Window cell of voxel j of slab s in the slab's z range [z0, z1), or -1.
// Every entry of slab s's bins lies in slab s, so along x (axis 0)
// j - s = nx (iy + ny iz) exactly and the cell iy + ny (iz - z0) is that
// quotient less ny z0 (an exact FP64 quotient, rounded); along y (axis 1)
// j - nx s = ix + nx ny iz and one exact integer division splits it.
__device__ __forceinline__ int window_cell(unsigned j, int axis, int s, int nlat, int z0, int z1, unsigned nx,
                                          unsigned nxy, double inv_nx, double inv_nxy)
{
    int cell;
    if (axis == 0) {
        cell = int(rint(double(j - unsigned(s)) * inv_nx)) - nlat * z0;
    } else {
        const unsigned rr = j - nx * unsigned(s);
        const unsigned iz = udiv_exact(rr, nxy, inv_nxy);
        cell = int(rr - iz * nxy) + nlat * (int(iz) - z0);
    }
    return cell >= 0 && cell < nlat * (z1 - z0) ? cell : -1;
}

__device__ __forceinline__ void window_add(unsigned long long *win, int cell, unsigned long long w)
{
    if (cell >= 0) atomicAdd(&win[cell], w);
}

__device__ __forceinline__ void slab_commit_body(const ProtonsDev &p, int64_t lo, int nb, const BinsDev &bins,
                                                 int par, unsigned long long *ovf, int *ovf_flag,
                                                 float *__restrict__ x, float *__restrict__ xlo, const GridDev &g,
                                                 int zc, int nzc, int comp, unsigned *status)
{
    extern __shared__ unsigned long long win[];
    const int tid = int(threadIdx.x);
    const int s = int(blockIdx.x) / nzc, zi = int(blockIdx.x) % nzc;
    if (zi == 0) {
        uint4 *c2 = reinterpret_cast<uint4 *>(bins.j0 + (size_t(1 - par) * bins.nslab + s) * bins.cap);
        for (int q = tid; q < bins.cap / 4; q += kSlabWG) c2[q] = make_uint4(kEmptyBin, kEmptyBin, kEmptyBin, kEmptyBin);
        if (s == 0 && tid == 0) ovf_flag[1 - par] = 0;
    }
    if (blockIdx.x == 0) {
        // every voxel's block sum is bounded by the sum over the rows of their
        // largest contribution: past kSumMax a sum may have left the word's range
        __shared__ double wsum[kSlabWG / 64];
        double t = 0.0;
        for (int q = tid; q < nb; q += kSlabWG) t += double(bins.rowmax[q]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if ((tid & 63) == 0) wsum[tid >> 6] = t;
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int w = 0; w < kSlabWG / 64; ++w) tot += wsum[w];
            if (!(tot < kSumMax)) atomicOr(status, PCT_DEV_ACC_RANGE);
        }
    }
    const int axis = block_axis(p, lo);
    if (s >= g.n[axis]) return;
    const int nlat = g.n[1 - axis];
    const int z0 = zi * zc, z1 = min(g.n[2], z0 + zc);
    if (z0 >= z1) return;
    const int nw = nlat * (z1 - z0);
    const unsigned *j0 = bins.j0 + (size_t(par) * bins.nslab + s) * bins.cap;
    const unsigned long long *w = bins.w + size_t(s) * kBinCap * bins.cap;
    const unsigned *j1 = bins.j1 + size_t(s) * (kBinCap - 1) * bins.cap;
    const int cap = bins.cap;
    const unsigned nx = unsigned(g.n[0]), nxy = unsigned(g.n[0]) * unsigned(g.n[1]);
    const double inv_nx = g.inv_n[0], inv_nxy = g.inv_nxy;
    unsigned jr[kRowsPerThread];
    unsigned long long wr[kRowsPerThread];
#pragma unroll
    for (int m = 0; m < kRowsPerThread; ++m) {
        const int r = tid + m * kSlabWG;
        jr[m] = kEmptyBin;
        wr[m] = 0ull;
        if (r < nb) {
            jr[m] = j0[r];
            wr[m] = w[r];
        }
    }
    // the further entries of the rows with two or more (one batch of loads)
    unsigned jb[kRowsPerThread][kBinCap - 1];
    unsigned long long wb[kRowsPerThread][kBinCap - 1];
#pragma unroll
    for (int m = 0; m < kRowsPerThread; ++m) {
        const int r = tid + m * kSlabWG;
#pragma unroll
        for (int k = 1; k < kBinCap; ++k) {
            jb[m][k - 1] = kEmptyBin;
            wb[m][k - 1] = 0ull;
            if (jr[m] != kEmptyBin && (jr[m] >> 30) >= unsigned(k)) {
                jb[m][k - 1] = j1[size_t(k - 1) * cap + r];
                wb[m][k - 1] = w[size_t(k) * cap + r];
            }
        }
    }
    // the window is cleared while the entries are in flight
    for (int q = tid; q < nw; q += kSlabWG) win[q] = 0ull;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kRowsPerThread; ++m) {
        if (jr[m] == kEmptyBin) continue;
        const int c = int(jr[m] >> 30) + 1;
        window_add(win, window_cell(jr[m] & 0x3FFFFFFFu, axis, s, nlat, z0, z1, nx, nxy, inv_nx, inv_nxy), wr[m]);
#pragma unroll
        for (int k = 1; k < kBinCap; ++k)
            if (k < c)
                window_add(win, window_cell(jb[m][k - 1], axis, s, nlat, z0, z1, nx, nxy, inv_nx, inv_nxy),
                           wb[m][k - 1]);
    }
    const bool of = ovf_flag[par] != 0;
    __syncthreads();
    const double inv_nlat = g.inv_n[1 - axis];
    for (int q0 = 0; q0 < nw; q0 += kCommitCells * kSlabWG) {
        int jv[kCommitCells];
        unsigned long long wv[kCommitCells];
        float xv[kCommitCells], lv[kCommitCells];
#pragma unroll
        for (int u = 0; u < kCommitCells; ++u) {
            const int q = q0 + tid + u * kSlabWG;
            jv[u] = -1;
            wv[u] = 0ull;
            if (q < nw) {
                const unsigned zq = udiv_exact(unsigned(q), unsigned(nlat), inv_nlat);
                const int a = q - int(zq) * nlat, zz = z0 + int(zq);
                const int ix = axis == 0 ? s : a, iy = axis == 0 ? a : s;
                jv[u] = ix + g.n[0] * (iy + g.n[1] * zz);
                wv[u] = win[q];
            }
        }
        if (of) {
#pragma unroll
            for (int u = 0; u < kCommitCells; ++u) {
                if (jv[u] >= 0) {
                    const unsigned long long o = ovf[jv[u]];
                    if (o != 0ull) {
                        wv[u] += o;
                        ovf[jv[u]] = 0ull;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kCommitCells; ++u) {
            xv[u] = 0.f;
            lv[u] = 0.f;
            if (wv[u] != 0ull) {
                xv[u] = x[jv[u]];
                if (comp) lv[u] = xlo[jv[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < kCommitCells; ++u) {
            if (wv[u] == 0ull) continue;
            if (comp) {
                int c;
                double sum;
                unpack_accumulator(wv[u], c, sum);
                const double v = double(xv[u]) + double(lv[u]) + sum / double(c);
                const float h = float(v);
                x[jv[u]] = h;
                xlo[jv[u]] = float(v - double(h));
            } else {
                x[jv[u]] = committed_value(xv[u], wv[u]);
            }
        }
    }
}

__global__ void __launch_bounds__(kSlabWG) k_slab_commit(ProtonsDev p, int64_t lo, int nb, BinsDev bins, int par,
                                                         unsigned long long *ovf, int *ovf_flag,
                                                         float *__restrict__ x, float *__restrict__ xlo, GridDev g,
                                                         int zc, int nzc, int comp, unsigned *status, GateDev gt)
{
    if (gate_closed(gt.halt)) return;
    slab_commit_body(p, lo, nb, bins, par, ovf, ovf_flag, x, xlo, g, zc, nzc, comp, status);
    gate_commit_end(gt);
}

// Commit of one block: a dense, coalesced scan of the block's touched index
// range; voxels with a non-zero row count get x_j += acc_j / s_j and are reset.
// Also re-arms the range words of the next block.
template <typename T>
__device__ __forceinline__ void drop_commit_body(T *x, void *accv, int32_t *cnt, const int *range_this,
                                                 int *range_next, long long *acc_lo)
{
    const int j0 = range_this[0], j1 = range_this[1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        range_next[0] = INT_MAX;
        range_next[1] = -1;
    }
    if (j1 < j0 || j0 < 0) return;  // nothing touched
    const int stride = int(gridDim.x * blockDim.x);
    if constexpr (sizeof(T) == 4) {
        // four 64-bit words per thread (the accumulator has 4 words of padding
        // past the last voxel; untouched words are zero)
        unsigned long long *pk = static_cast<unsigned long long *>(accv);
        for (int j = (j0 & ~3) + 4 * int(blockIdx.x * blockDim.x + threadIdx.x); j <= j1; j += 4 * stride) {
            const ulonglong2 w01 = *reinterpret_cast<const ulonglong2 *>(pk + j);
            const ulonglong2 w23 = *reinterpret_cast<const ulonglong2 *>(pk + j + 2);
            const unsigned long long w[4] = {w01.x, w01.y, w23.x, w23.y};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (w[e] != 0ull) {
                    int c;
                    double sum;
                    unpack_accumulator(w[e], c, sum);
                    if (c > 0) x[j + e] = T(double(x[j + e]) + sum / double(c));
                    pk[j + e] = 0ull;
                }
            }
        }
        return;
    }
    for (int j = j0 + int(blockIdx.x * blockDim.x + threadIdx.x); j <= j1; j += stride) {
        {
            const int c = cnt[j];
            if (c != 0) {
                if (acc_lo) {
                    long long *hi = static_cast<long long *>(accv);
                    x[j] = T(double(x[j]) + det_sum(hi[j], acc_lo[j]) / double(c));
                    hi[j] = 0;
                    acc_lo[j] = 0;
                } else {
                    double *acc = static_cast<double *>(accv);
                    x[j] = T(double(x[j]) + acc[j] / double(c));
                    acc[j] = 0.0;
                }
                cnt[j] = 0;
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_drop_commit(T *x, void *accv, int32_t *cnt, const int *range_this,
                                                     int *range_next, long long *acc_lo, GateDev gt)
{
    if (gate_closed(gt.halt)) return;
    drop_commit_body<T>(x, accv, cnt, range_this, range_next, acc_lo);
    gate_commit_end(gt);
}

__global__ void k_reset_ranges(int *hdr)
{
    if (threadIdx.x == 0) {
        hdr[kHdrRange0] = INT_MAX;
        hdr[kHdrRange0 + 1] = -1;
        hdr[kHdrRange1] = INT_MAX;
        hdr[kHdrRange1 + 1] = -1;
    }
}

// ---------------------------------------------------------------------------
// total variation
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double tv_diffs(const T *__restrict__ x, const GridDev &g, int ix, int iy, int iz,
                                           int64_t v, double eps, double &dx, double &dy, double &dz)
{
    const int64_t sy = g.n[0], sz = int64_t(g.n[0]) * g.n[1];
    double xv = x[v];
    dx = ix + 1 < g.n[0] ? double(x[v + 1]) - xv : 0.0;
    dy = iy + 1 < g.n[1] ? double(x[v + sy]) - xv : 0.0;
    dz = iz + 1 < g.n[2] ? double(x[v + sz]) - xv : 0.0;
    return sqrt(dx * dx + dy * dy + dz * dz + eps * eps);
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_tv(const T *__restrict__ x, GridDev g, double eps, T *grad,
                                            double *partial, int64_t nvox)
{
    __shared__ double red[kWG];
    double local = 0.0;
    const int64_t sy = g.n[0], sz = int64_t(g.n[0]) * g.n[1];
    for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nvox; v += int64_t(gridDim.x) * blockDim.x) {
        int ix = int(v % g.n[0]);
        int iy = int((v / g.n[0]) % g.n[1]);
        int iz = int(v / sz);
        double dx, dy, dz;
        double s = tv_diffs(x, g, ix, iy, iz, v, eps, dx, dy, dz);
        local += s;
        if (grad) {
            double gv = -(dx + dy + dz) / s;
            double ex, ey, ez;
            if (ix > 0) gv += (double(x[v]) - double(x[v - 1])) / tv_diffs(x, g, ix - 1, iy, iz, v - 1, eps, ex, ey, ez);
            if (iy > 0) gv += (double(x[v]) - double(x[v - sy])) / tv_diffs(x, g, ix, iy - 1, iz, v - sy, eps, ex, ey, ez);
            if (iz > 0) gv += (double(x[v]) - double(x[v - sz])) / tv_diffs(x, g, ix, iy, iz - 1, v - sz, eps, ex, ey, ez);
            grad[v] = T(gv);
        }
    }
    red[threadIdx.x] = local;
    __syncthreads();
    for (int s = kWG / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kWG) k_sum_partials(const double *__restrict__ partial, int n, double *out)
{
    __shared__ double red[kWG];
    double local = 0.0;
    for (int q = threadIdx.x; q < n; q += kWG) local += partial[q];
    red[threadIdx.x] = local;
    __syncthreads();
    for (int s = kWG / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// ---------------------------------------------------------------------------
// region selection (Algorithm 1, step 2): stable compaction of the records
// whose entry and exit slices lie in [z_lo, z_hi].  Each of G workgroups owns
// a contiguous chunk of the input: count, exclusive scan of the G counts,
// then an ordered scatter (wave ballots) inside every chunk.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int slice_index(float v, const GridDev &g)
{
    const double d = double(v);
    if (!isfinite(d)) return -1;
    const double s = floor((d - g.lo[2]) / g.pitch[2]);
    return int(fmin(fmax(s, 0.0), double(g.n[2] - 1)));
}

__device__ __forceinline__ bool region_member(const ProtonsDev &p, int64_t i, const GridDev &g, int z_lo, int z_hi)
{
    const int a = slice_index(p.v_in[i], g);
    const int c = slice_index(p.v_out[i], g);
    return a >= z_lo && a <= z_hi && c >= z_lo && c <= z_hi;
}

constexpr int kSelWG = 256;

// histogram of |exit slice - entry slice|: LDS bins per workgroup, then one
// global atomic per non-empty bin
__global__ void __launch_bounds__(kSelWG) k_span_histogram(ProtonsDev p, int64_t n, GridDev g,
                                                            unsigned long long *hist)
{
    extern __shared__ unsigned int bins[];
    const int nz = g.n[2];
    for (int k = threadIdx.x; k < nz; k += kSelWG) bins[k] = 0u;
    __syncthreads();
    for (int64_t i = int64_t(blockIdx.x) * kSelWG + threadIdx.x; i < n; i += int64_t(gridDim.x) * kSelWG) {
        const int a = slice_index(p.v_in[i], g);
        const int c = slice_index(p.v_out[i], g);
        if (a >= 0 && c >= 0) atomicAdd(&bins[a > c ? a - c : c - a], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nz; k += kSelWG)
        if (bins[k]) atomicAdd(hist + k, static_cast<unsigned long long>(bins[k]));
}

__global__ void __launch_bounds__(kSelWG) k_region_count(ProtonsDev p, int64_t n, int64_t chunk, GridDev g,
                                                          int z_lo, int z_hi, long long *partial)
{
    __shared__ long long red[kSelWG / 64];
    const int64_t a = int64_t(blockIdx.x) * chunk;
    const int64_t e = min(n, a + chunk);
    long long c = 0;
    for (int64_t i = a + threadIdx.x; i < e; i += kSelWG) c += region_member(p, i, g, z_lo, z_hi) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < kSelWG / 64; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

// exclusive scan of G <= kMaxPartials counts in place; total to *count
__global__ void __launch_bounds__(kSelWG) k_region_scan(long long *partial, int G, int64_t *count)
{
    __shared__ long long run[kSelWG];
    const int per = (G + kSelWG - 1) / kSelWG;
    const int a = int(threadIdx.x) * per;
    const int e = min(G, a + per);
    long long s = 0;
    for (int k = a; k < e; ++k) s += partial[k];
    run[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long acc = 0;
        for (int t = 0; t < kSelWG; ++t) {
            const long long v = run[t];
            run[t] = acc;
            acc += v;
        }
        if (count) *count = acc;
    }
    __syncthreads();
    long long acc = run[threadIdx.x];
    for (int k = a; k < e; ++k) {
        const long long v = partial[k];
        partial[k] = acc;
        acc += v;
    }
}

__global__ void __launch_bounds__(kSelWG) k_region_scatter(ProtonsDev p, const float *b, int64_t n, int64_t chunk,
                                                            GridDev g, int z_lo, int z_hi, const long long *partial,
                                                            ProtonsBufDev out, int64_t capacity, float *b_out)
{
    __shared__ int wave_cnt[kSelWG / 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t a = int64_t(blockIdx.x) * chunk;
    const int64_t e = min(n, a + chunk);
    long long base = partial[blockIdx.x];
    for (int64_t t0 = a; t0 < e; t0 += kSelWG) {
        const int64_t i = t0 + threadIdx.x;
        const bool f = i < e && region_member(p, i, g, z_lo, z_hi);
        const unsigned long long mask = __ballot(f);
        if (lane == 0) wave_cnt[wave] = __popcll(mask);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < kSelWG / 64; ++w) {
            before += w < wave ? wave_cnt[w] : 0;
            total += wave_cnt[w];
        }
        const long long dst = base + before + __popcll(mask & ((1ull << lane) - 1ull));
        if (f && dst < capacity) {
            out.t_in[dst] = p.t_in[i];
            out.v_in[dst] = p.v_in[i];
            out.th_in[dst] = p.th_in[i];
            out.ph_in[dst] = p.ph_in[i];
            out.t_out[dst] = p.t_out[i];
            out.v_out[dst] = p.v_out[i];
            out.th_out[dst] = p.th_out[i];
            out.ph_out[dst] = p.ph_out[i];
            out.gantry[dst] = p.gantry[i];
            if (b_out) b_out[dst] = b[i];
        }
        base += total;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// stored rows (precision form): trace once, sweep from the stored CSR rows
// ---------------------------------------------------------------------------
// Counting sink: merged pieces of a row.
struct CountSink {
    int32_t n;
    __device__ __forceinline__ void segment(double, double) {}
    __device__ __forceinline__ void final(int, int, int, int, double) { ++n; }
};

// Row lengths (after consecutive merge) into offsets[1..n].
template <bool HULL>
__global__ void __launch_bounds__(kWG) k_row_lengths(ProtonsDev p, int64_t n, long long *len_out,
                                                     const PathSrc src,  GridDev g,
                                                     unsigned *status)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Rec r = load_rec(p, i);
    CountSink cs{0};
    if (rec_finite(r)) {
        Merge<CountSink, PCT_CHORD_F64> m(cs, g);
        walk_path<HULL>(r, src, g, m);
        m.finish();
    } else {
        raise_status(status, PCT_DEV_NONFINITE);
    }
    len_out[i] = cs.n;
}

// chunk sums of v[0..n) (G chunks of `chunk` values)
__global__ void __launch_bounds__(kSelWG) k_chunk_sums(const long long *v, int64_t n, int64_t chunk,
                                                        long long *partial)
{
    __shared__ long long red[kSelWG / 64];
    const int64_t a = int64_t(blockIdx.x) * chunk;
    const int64_t e = min(n, a + chunk);
    long long c = 0;
    for (int64_t i = a + threadIdx.x; i < e; i += kSelWG) c += v[i];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < kSelWG / 64; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

// in-place inclusive scan of every chunk, offset by the chunk's exclusive base
__global__ void __launch_bounds__(kSelWG) k_chunk_scan(long long *v, int64_t n, int64_t chunk,
                                                        const long long *partial)
{
    __shared__ long long tile[kSelWG];
    const int64_t a = int64_t(blockIdx.x) * chunk;
    const int64_t e = min(n, a + chunk);
    long long base = partial[blockIdx.x];
    for (int64_t t0 = a; t0 < e; t0 += kSelWG) {
        const int64_t i = t0 + threadIdx.x;
        tile[threadIdx.x] = i < e ? v[i] : 0;
        __syncthreads();
        for (int d = 1; d < kSelWG; d <<= 1) {
            const long long add = int(threadIdx.x) >= d ? tile[threadIdx.x - d] : 0;
            __syncthreads();
            tile[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < e) v[i] = base + tile[threadIdx.x];
        base += tile[kSelWG - 1];
        __syncthreads();
    }
}

// Stored chord formats.
template <int CT>
struct StoredChord;
template <>
struct StoredChord<PCT_CHORD_F32> {
    using type = float;
    __device__ static __forceinline__ float put(double c) { return float(c); }
    __device__ static __forceinline__ float get(float v) { return v; }
};
template <>
struct StoredChord<PCT_CHORD_F16> {
    using type = unsigned short;
    __device__ static __forceinline__ unsigned short put(double c)
    {
        // c is already an FP16 value: the conversion is exact
        return __half_as_ushort(__float2half(float(c)));
    }
    __device__ static __forceinline__ float get(unsigned short v) { return __half2float(__ushort_as_half(v)); }
};
template <>
struct StoredChord<PCT_CHORD_BF16> {
    using type = unsigned short;
    __device__ static __forceinline__ unsigned short put(double c)
    {
        // c is already a BF16 value: its float has 16 zero low bits
        return static_cast<unsigned short>(__float_as_uint(float(c)) >> 16);
    }
    __device__ static __forceinline__ float get(unsigned short v) { return __uint_as_float(unsigned(v) << 16); }
};

template <int CT>
struct RowSink {
    using S = StoredChord<CT>;
    int32_t *vox;
    typename S::type *ch;
    int64_t pos, end;
    Reentry re;
    double n2;
    __device__ __forceinline__ void segment(double dx, double dy) { re.segment(dx, dy); }
    __device__ __forceinline__ void final(int j, int ix, int iy, int iz, double c)
    {
        bool first;
        const double aprev = re.visit(j, ix, iy, iz, c, first);
        n2 += c * (2.0 * aprev + c);
        if (pos < end) {
            vox[pos] = first ? int(unsigned(j) | 0x80000000u) : j;
            ch[pos] = S::put(c);
        }
        ++pos;
    }
};

template <int CT, bool HULL>
__global__ void __launch_bounds__(kWG) k_rows_build(ProtonsDev p, int64_t n, const long long *__restrict__ offsets,
                                                    int32_t *vox, typename StoredChord<CT>::type *chord, double *n2,
                                                    const PathSrc src,  GridDev g,
                                                    unsigned *status)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Rec r = load_rec(p, i);
    RowSink<CT> rs{vox, chord, offsets[i], offsets[i + 1], {}, 0.0};
    rs.re.init(r);
    if (rec_finite(r)) {
        Merge<RowSink<CT>, CT> m(rs, g);
        walk_path<HULL>(r, src, g, m);
        m.finish();
        if (rs.re.unsafe) raise_status(status, PCT_DEV_REENTRY);
    } else {
        raise_status(status, PCT_DEV_NONFINITE);
    }
    if (rs.pos != rs.end) raise_status(status, PCT_DEV_ROW_OVERFLOW);  // offsets from other records
    n2[i] = rs.n2;
}

struct RowsDev {
    const long long *offsets;
    const int32_t *vox;
    const void *chord;
    const double *n2;
};

constexpr int kRowRegs = 8;  // pieces per lane kept in registers between the gather and the scatter

// Fused FP32 DROP block over stored rows: LPR lanes per row, 64 / LPR rows per
// one-wave workgroup; commit workgroups first (see k_drop_fused).
template <int CT, int LPR>
__global__ void __launch_bounds__(64) k_drop_rows_fused(RowsDev rows, const float *__restrict__ b,
                                                        const float *__restrict__ base, float *__restrict__ next,
                                                        const unsigned long long *__restrict__ pk_prev,
                                                        unsigned long long *pk_cur, unsigned long long *pk_old,
                                                        int *r_cur, const int *r_prev, const int *r_old,
                                                        int *r_reset, int64_t lo, int64_t hi, double lambda,
                                                        unsigned *status, int nvox)
{
    if (int(blockIdx.x) < kCommitWG) {
        commit_part(base, next, pk_prev, pk_old, r_prev, r_old, r_reset, nvox, int(blockIdx.x), kCommitWG);
        return;
    }
    using S = StoredChord<CT>;
    const typename S::type *__restrict__ chord = static_cast<const typename S::type *>(rows.chord);
    constexpr int RPW = 64 / LPR;
    const int lane = threadIdx.x;
    const int l = lane % LPR;
    const int64_t i = lo + int64_t(blockIdx.x - kCommitWG) * RPW + lane / LPR;
    bool active = i < hi;
    int64_t a = 0, e = 0;
    double bi = 0.0, n2 = 0.0;
    if (active) {
        a = rows.offsets[i];
        e = rows.offsets[i + 1];
        bi = double(b[i]);
        n2 = rows.n2[i];
        if (!isfinite(bi)) {
            if (l == 0) raise_status(status, PCT_DEV_NONFINITE);
            active = false;
        }
    }
    if (!active) e = a;
    const LazyX xa{base, pk_prev};
    int jr[kRowRegs];
    float cr[kRowRegs];
    double dot = 0.0;
    // a piece naming a voxel outside the grid (rows built for another
    // plan) is dropped: chord 0 and voxel 0
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kRowRegs; ++k) {
        const int64_t q = a + l + int64_t(k) * LPR;
        jr[k] = 0;
        cr[k] = 0.f;
        if (q < e) {
            const int v = rows.vox[q];
            if ((v & 0x7FFFFFFF) < nvox) {
                jr[k] = v;
                cr[k] = S::get(chord[q]);
            } else {
                bad = true;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kRowRegs; ++k)
        if (a + l + int64_t(k) * LPR < e) dot += double(cr[k]) * xa(jr[k] & 0x7FFFFFFF);
    for (int64_t q = a + l + int64_t(kRowRegs) * LPR; q < e; q += LPR) {
        const int j = rows.vox[q] & 0x7FFFFFFF;
        if (j < nvox)
            dot += double(S::get(chord[q])) * xa(j);
        else
            bad = true;
    }
    if (bad) raise_status(status, PCT_DEV_BAD_ROW);
    dot = group_sum<LPR>(dot);
    int jmin = INT_MAX, jmax = -1;
    if (active && n2 > 0.0) {
        const double rho = lambda * (bi - dot) / n2;
#pragma unroll
        for (int k = 0; k < kRowRegs; ++k) {
            if (a + l + int64_t(k) * LPR < e) {
                const int j = jr[k] & 0x7FFFFFFF;
                atomicAdd(pk_cur + j, pack_contribution(rho * double(cr[k]), jr[k] < 0, status));
                jmin = min(jmin, j);
                jmax = max(jmax, j);
            }
        }
        for (int64_t q = a + l + int64_t(kRowRegs) * LPR; q < e; q += LPR) {
            const int v = rows.vox[q];
            const int j = v & 0x7FFFFFFF;
            if (j >= nvox) continue;
            atomicAdd(pk_cur + j, pack_contribution(rho * double(S::get(chord[q])), v < 0, status));
            jmin = min(jmin, j);
            jmax = max(jmax, j);
        }
    }
    publish_range(jmin, jmax, r_cur);
}

// ---------------------------------------------------------------------------
// within-block ordering: every block of consecutive records is sorted by
// (entry slice, t_in, input position) with a bitonic sort of packed 64-bit
// keys in LDS, one workgroup per block
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long order_key(const ProtonsDev &p, int64_t i, int local, const GridDev &g)
{
    const unsigned slice = unsigned(slice_index(p.v_in[i], g) + 1);  // 0 for a non-finite v_in
    unsigned t = __float_as_uint(p.t_in[i]);
    t ^= (t & 0x80000000u) ? 0xFFFFFFFFu : 0x80000000u;               // order-preserving bits
    return (static_cast<unsigned long long>(slice & 0xFFFFu) << 48) | (static_cast<unsigned long long>(t) << 16) |
           static_cast<unsigned long long>(local);
}

__global__ void __launch_bounds__(kSelWG) k_order_blocks(ProtonsDev p, const float *b, int64_t n, int64_t block,
                                                          int p2, GridDev g, ProtonsBufDev out, float *b_out)
{
    extern __shared__ unsigned long long keys[];
    const int64_t lo = int64_t(blockIdx.x) * block;
    const int cnt = int(min(block, n - lo));
    for (int q = threadIdx.x; q < p2; q += kSelWG) keys[q] = q < cnt ? order_key(p, lo + q, q, g) : ~0ull;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int q = threadIdx.x; q < p2; q += kSelWG) {
                const int r = q ^ j;
                if (r > q) {
                    const unsigned long long a = keys[q], c = keys[r];
                    const bool up = (q & k) == 0;
                    if ((a > c) == up) {
                        keys[q] = c;
                        keys[r] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int q = threadIdx.x; q < cnt; q += kSelWG) {
        const int64_t src = lo + int64_t(keys[q] & 0xFFFFull);
        const int64_t dst = lo + q;
        out.t_in[dst] = p.t_in[src];
        out.v_in[dst] = p.v_in[src];
        out.th_in[dst] = p.th_in[src];
        out.ph_in[dst] = p.ph_in[src];
        out.t_out[dst] = p.t_out[src];
        out.v_out[dst] = p.v_out[src];
        out.th_out[dst] = p.th_out[src];
        out.ph_out[dst] = p.ph_out[src];
        out.gantry[dst] = p.gantry[src];
        if (b_out) b_out[dst] = b[src];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline char *wsb(void *ws) { return static_cast<char *>(ws); }

static inline unsigned grid_for(int64_t n) { return unsigned((n + kWG - 1) / kWG); }

int upload_table(const pct_plan &pl, void *ws, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    hipError_t e = hipMemcpyAsync(wsb(ws) + L.table, pl.table.data(), pl.table.size() * sizeof(double),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(wsb(ws) + L.hdr, 0, 256, s);
    if (e != hipSuccess) return e;
    // the DROP accumulators and row counts start at zero; every block leaves
    // them at zero again
    e = hipMemsetAsync(wsb(ws) + L.acc, 0, L.cnt - L.acc, s);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(wsb(ws) + L.cnt, 0, size_t(pl.nvox) * sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

int read_status(const pct_plan &pl, void *ws, int reset, uint32_t *bits, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, wsb(ws) + L.hdr, sizeof(v), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    *bits = v;
    if (reset) {
        e = hipMemsetAsync(wsb(ws) + L.hdr, 0, sizeof(uint32_t), s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
    }
    return e;
}

static GateDev gate_dev(void *ws, const Layout &L, bool on)
{
    int *hdr = reinterpret_cast<int *>(wsb(ws) + L.hdr);
    GateDev gt{};
    if (!on) return gt;
    gt.halt = hdr + kHdrHalt;
    gt.wg_done = reinterpret_cast<unsigned *>(hdr + kHdrGateCount);
    gt.cancel = hdr + kHdrCancel;
    gt.done = reinterpret_cast<long long *>(hdr + kHdrDone);
    gt.status = reinterpret_cast<unsigned *>(hdr + kHdrStatus);
    return gt;
}

int write_cancel(pct_plan &pl, void *ws, int32_t request)
{
    hipStream_t cs = nullptr;
    {
        std::lock_guard<std::mutex> lock(pl.mu);
        if (!pl.cancel_stream) {
            hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
            if (e != hipSuccess) return e;
            pl.cancel_stream = cs;
        }
        cs = static_cast<hipStream_t>(pl.cancel_stream);
    }
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    int *word = reinterpret_cast<int *>(wsb(ws) + L.hdr) + kHdrCancel;
    hipError_t e = hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(word), request != 0 ? 1 : 0, 1, cs);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(cs);
}

int read_progress(const pct_plan &pl, void *ws, int64_t *done, int *halted, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    int32_t h[kHdrDone + 2];
    hipError_t e = hipMemcpyAsync(h, wsb(ws) + L.hdr, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    int64_t d;
    std::memcpy(&d, h + kHdrDone, sizeof(d));
    *done = d;
    *halted = h[kHdrHalt] != 0;
    return hipSuccess;
}

int launch_gate_reset(const pct_plan &pl, void *ws, void *stream)
{
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    hipLaunchKernelGGL(k_gate_begin, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), gate_dev(ws, L, true));
    return hipGetLastError();
}

int launch_trace(const pct_plan &pl, const ProtonsDev &p, int64_t first, int64_t count, int32_t max_nnz,
                 int32_t *vox, double *chord, int32_t *nnz, void *ws, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    const PathSrc src = path_src(pl, wsb(ws) + L.table);
    unsigned *status = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr) + kHdrStatus;
    if (src.hull)
        hipLaunchKernelGGL(k_trace<true>, dim3(grid_for(count)), dim3(kWG), 0, s, p, first, count, max_nnz, vox,
                           chord, nnz, src, grid_dev(pl.grid), status);
    else
        hipLaunchKernelGGL(k_trace<false>, dim3(grid_for(count)), dim3(kWG), 0, s, p, first, count, max_nnz, vox,
                           chord, nnz, src, grid_dev(pl.grid), status);
    return hipGetLastError();
}

// Launches of the one-lane-per-proton kernels, in pieces of at most 2^30
// workgroups (protons [first, first + count) per piece).
template <class F>
static void launch_pieces(int64_t n, F &&piece)
{
    const int64_t max_n = int64_t(kWG) << 30;
    for (int64_t first = 0; first < n; first += max_n) piece(first, std::min<int64_t>(n - first, max_n));
}

int launch_forward(const pct_plan &pl, const ProtonsDev &p, int64_t n, const void *x, int dtype, void *y,
                   void *nrm2, void *ws, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    const PathSrc src = path_src(pl, wsb(ws) + L.table);
    unsigned *status = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr) + kHdrStatus;
    GridDev g = grid_dev(pl.grid);
    auto go = [&](auto hull) {
        constexpr bool H = decltype(hull)::value;
        launch_pieces(n, [&](int64_t first, int64_t cnt) {
            if (dtype == PCT_F64)
                hipLaunchKernelGGL((k_forward<double, H>), dim3(grid_for(cnt)), dim3(kWG), 0, s, p, first,
                                   first + cnt, static_cast<const double *>(x), static_cast<double *>(y),
                                   static_cast<double *>(nrm2), src, g, status);
            else
                hipLaunchKernelGGL((k_forward<float, H>), dim3(grid_for(cnt)), dim3(kWG), 0, s, p, first,
                                   first + cnt, static_cast<const float *>(x), static_cast<float *>(y),
                                   static_cast<float *>(nrm2), src, g, status);
        });
    };
    if (src.hull)
        go(std::true_type{});
    else
        go(std::false_type{});
    return hipGetLastError();
}

int launch_backproject(const pct_plan &pl, const ProtonsDev &p, int64_t n, const void *r, int dtype, void *gout,
                       void *ws, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    const PathSrc src = path_src(pl, wsb(ws) + L.table);
    unsigned *status = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr) + kHdrStatus;
    GridDev g = grid_dev(pl.grid);
    auto go = [&](auto hull) {
        constexpr bool H = decltype(hull)::value;
        launch_pieces(n, [&](int64_t first, int64_t cnt) {
            if (dtype == PCT_F64)
                hipLaunchKernelGGL((k_backproject<double, H>), dim3(grid_for(cnt)), dim3(kWG), 0, s, p, first,
                                   first + cnt, static_cast<const double *>(r), static_cast<double *>(gout), src,
                                   g, status);
            else
                hipLaunchKernelGGL((k_backproject<float, H>), dim3(grid_for(cnt)), dim3(kWG), 0, s, p, first,
                                   first + cnt, static_cast<const float *>(r), static_cast<float *>(gout), src, g,
                                   status);
        });
    };
    if (src.hull)
        go(std::true_type{});
    else
        go(std::false_type{});
    return hipGetLastError();
}

// Profiling: a pool of event pairs per kernel kind; launches are sampled
// evenly so that at most kProfSamples pairs are recorded per call.
constexpr int kProfSamples = 512;

static hipError_t prof_prepare(pct_plan &pl)
{
    for (int k = 0; k < 2; ++k) {
        pl.prof_used[k] = 0;
        while (pl.prof_events[k].size() < size_t(2 * kProfSamples)) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            pl.prof_events[k].push_back(e);
        }
    }
    return hipSuccess;
}

static inline hipEvent_t prof_event(pct_plan &pl, int kind, int idx)
{
    return static_cast<hipEvent_t>(pl.prof_events[kind][idx]);
}

int profile_read(pct_plan &pl, double ms[2], int64_t launches[2])
{
    for (int k = 0; k < 2; ++k) {
        ms[k] = 0.0;
        launches[k] = pl.prof_used[k];
        for (int i = 0; i < pl.prof_used[k]; ++i) {
            hipEvent_t a = prof_event(pl, k, 2 * i), b = prof_event(pl, k, 2 * i + 1);
            hipError_t e = hipEventSynchronize(b);
            if (e != hipSuccess) return e;
            float t = 0.f;
            e = hipEventElapsedTime(&t, a, b);
            if (e != hipSuccess) return e;
            ms[k] += t;
        }
    }
    return hipSuccess;
}

void profile_release(pct_plan &pl)
{
    for (int k = 0; k < 2; ++k) {
        for (void *e : pl.prof_events[k]) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
        pl.prof_events[k].clear();
        pl.prof_used[k] = 0;
    }
}

// Launch of one block's fused kernel with the chosen lanes per proton.
template <typename T, int CHORD, bool HULL>
static void launch_block(int lanes, hipStream_t s, const ProtonsDev &p, const float *b, T *x, void *acc, int32_t *cnt,
                         int *range, const PathSrc &src, const GridDev &g, int64_t lo, int64_t hi,
                         double lambda, unsigned *status, long long *acc_lo, const int *halt)
{
    const int64_t n = hi - lo;
    switch (lanes) {
#define PCT_LAUNCH_LPP(LPP)                                                                                      \
    case LPP: {                                                                                                  \
        if constexpr (!HULL || LPP == 64) {                                                                      \
            const unsigned grid = unsigned((n + (64 / LPP) - 1) / (64 / LPP));                                \
            const size_t lds = size_t(64 / LPP) * kStageDoubles<HULL> * size_t(src.nvmax) * sizeof(double) + stash_bytes<T>(); \
            hipLaunchKernelGGL((k_drop_block<T, CHORD, LPP, HULL>), dim3(grid), dim3(64), lds, s, p, b, x, acc, \
                               cnt, range, src, g, lo, hi, lambda, status, acc_lo, halt);                       \
        }                                                                                                        \
        break;                                                                                                   \
    }
        PCT_LAUNCH_LPP(8)
        PCT_LAUNCH_LPP(16)
        PCT_LAUNCH_LPP(32)
        PCT_LAUNCH_LPP(64)
#undef PCT_LAUNCH_LPP
    default:
        hipLaunchKernelGGL((k_drop_rows<T, CHORD, HULL>), dim3(grid_for(n)), dim3(kWG), 0, s, p, b, x, acc, cnt,
                           range, src, g, lo, hi, lambda, status, acc_lo, halt);
    }
}

// Launch q of a fused FP32 sweep (see k_drop_fused): commit workgroups first,
// then the proton workgroups of block [lo, hi).
template <int CHORD, bool HULL>
static void launch_fused(int lanes, hipStream_t s, const ProtonsDev &p, const float *b, const float *base,
                         float *next, const unsigned long long *pk_prev, unsigned long long *pk_cur,
                         unsigned long long *pk_old, int *r_cur, const int *r_prev, const int *r_old, int *r_reset,
                         const PathSrc &src, const GridDev &g, int64_t lo, int64_t hi, double lambda,
                         unsigned *status, int nvox, int full)
{
    const int64_t n = hi - lo;
    switch (lanes) {
#define PCT_LAUNCH_FUSED(LPP)                                                                                    \
    case LPP: {                                                                                                  \
        if constexpr (!HULL || LPP == 64) {                                                                      \
            const int64_t n_wg = (n + (64 / LPP) - 1) / (64 / LPP);                                          \
            const unsigned grid = unsigned(kCommitWG + 8 * ((n_wg + 7) / 8));                                \
            const size_t lds = size_t(64 / LPP) * 3 * size_t(src.nvmax) * sizeof(double) + stash_bytes<float>(); \
            hipLaunchKernelGGL((k_drop_fused<CHORD, LPP, HULL>), dim3(grid), dim3(64), lds, s, p, b, base, next, \
                               pk_prev, pk_cur, pk_old, r_cur, r_prev, r_old, r_reset, src, g, lo, hi, lambda,  \
                               status, nvox, full);                                                              \
        }                                                                                                        \
        break;                                                                                                   \
    }
        PCT_LAUNCH_FUSED(8)
        PCT_LAUNCH_FUSED(16)
        PCT_LAUNCH_FUSED(32)
        PCT_LAUNCH_FUSED(64)
#undef PCT_LAUNCH_FUSED
    default: break;
    }
}

static_assert(kRowsPerThread * kSlabWG >= kBinMaxRows, "slab commit covers the largest binned block");

// Packed words of a slab-commit window: 128 KB of LDS once the kernel is
// allowed that much dynamic LDS, else 64 KB.
static int slab_window_words()
{
    static const int words = [] {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_slab_commit),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 int(kWinWords * sizeof(unsigned long long)));
        (void)hipGetLastError();
        return e == hipSuccess ? kWinWords : kWinWords / 2;
    }();
    return words;
}

// Launch of block [lo, hi) of the binned schedule (see k_drop_bin).
// With ev0/ev1 the launch records its own start and end in those events
// (profiling: no extra stream packets around the kernel).
template <int CHORD, bool HULL>
static void launch_bin(int lanes, hipStream_t s, const ProtonsDev &p, const float *b, const float *x,
                       const BinsDev &bins, int par, unsigned long long *ovf, int *ovf_flag, const PathSrc &src,
                       const GridDev &g, int64_t lo, int64_t hi, double lambda, unsigned *status,
                       const int *halt, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    const int64_t n = hi - lo;
    switch (lanes) {
#define PCT_LAUNCH_BIN(LPP)                                                                                      \
    case LPP: {                                                                                                  \
        if constexpr (!HULL || LPP == 64) {                                                                      \
            const int64_t n_wg = (n + (64 / LPP) - 1) / (64 / LPP);                                          \
            const unsigned grid = unsigned(8 * ((n_wg + 7) / 8));                                            \
            const size_t lds = size_t(64 / LPP) * kStageDoubles<HULL> * size_t(src.nvmax) * sizeof(double) + \
                               stash_bytes<float>();                                                      \
            if (ev0)                                                                                             \
                hipExtLaunchKernelGGL((k_drop_bin<CHORD, LPP, HULL>), dim3(grid), dim3(64), uint32_t(lds), s, ev0, \
                                      ev1, 0u, p, b, x, bins, par, ovf, ovf_flag, src, g, lo, hi, lambda, status, \
                                      halt);                                                                     \
            else                                                                                                 \
                hipLaunchKernelGGL((k_drop_bin<CHORD, LPP, HULL>), dim3(grid), dim3(64), lds, s, p, b, x, bins,  \
                                   par, ovf, ovf_flag, src, g, lo, hi, lambda, status, halt);                   \
        }                                                                                                        \
        break;                                                                                                   \
    }
        PCT_LAUNCH_BIN(8)
        PCT_LAUNCH_BIN(16)
        PCT_LAUNCH_BIN(32)
        PCT_LAUNCH_BIN(64)
#undef PCT_LAUNCH_BIN
    default: break;
    }
}

// Lanes per proton: enough lanes that each walks a few slabs of the dominant
// axis, within the LDS budget of the staged vertex coordinates.
constexpr int64_t kPipeMaxBlock = 4096;

static int choose_lanes(const pct_plan &pl, int requested)
{
    constexpr size_t kLdsBudget = 64 * 1024;
    int lanes = requested;
    if (lanes == 0) {
        const int ndom = std::max(pl.grid.nx, pl.grid.ny);
        lanes = ndom >= 160 ? 64 : ndom >= 64 ? 32 : 16;
    }
    if (pl.hull && lanes != 1) lanes = 64;  // the hull instantiations use 64 lanes per proton
    if (lanes > 1 && size_t(64 / lanes) * 3 * size_t(path_vertices_max(pl)) * sizeof(double) + stash_bytes<double>() >
                         kLdsBudget)
        lanes = 1;
    return lanes;
}

void graph_release(pct_plan &pl)
{
    if (pl.graph_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(pl.graph_exec));
    pl.graph_exec = nullptr;
    pl.graph_key.clear();
    if (pl.capture_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(pl.capture_stream));
    pl.capture_stream = nullptr;
    if (pl.cancel_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(pl.cancel_stream));
    pl.cancel_stream = nullptr;
}

// Buffers of the fused FP32 schedule: X[0] = x, X[1] in the workspace,
// accumulators PK[0..2], range slots R[0..3] (header words from kHdrSlots).
struct FusedBufs {
    float *X[2];
    unsigned long long *PK[3];
    int *R[4];
    int nv;
    unsigned copy_grid;
};

static FusedBufs fused_bufs(const pct_plan &pl, void *ws, float *x)
{
    const Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    FusedBufs F;
    F.X[0] = x;
    F.X[1] = reinterpret_cast<float *>(wsb(ws) + L.x1);
    for (int k = 0; k < 3; ++k)
        F.PK[k] = reinterpret_cast<unsigned long long *>(wsb(ws) + L.acc + size_t(k) * L.acc_stride);
    int *hdr = reinterpret_cast<int *>(wsb(ws) + L.hdr);
    for (int k = 0; k < 4; ++k) F.R[k] = hdr + kHdrSlots + 2 * k;
    F.nv = int(pl.nvox);
    F.copy_grid = unsigned(std::min<int64_t>(2048, (pl.nvox + 255) / 256));
    return F;
}

// Arguments of the launch at position q of a fused sweep (see k_drop_fused).
struct FusedStep {
    const float *base;
    float *next;
    const unsigned long long *pk_prev;
    unsigned long long *pk_cur, *pk_old;
    int *r_cur;
    const int *r_prev, *r_old;
    int *r_reset;
};

static FusedStep fused_step(const FusedBufs &F, int64_t q)
{
    return FusedStep{F.X[q % 2],       F.X[(q + 1) % 2], F.PK[(q + 2) % 3], F.PK[q % 3],      F.PK[(q + 1) % 3],
                     F.R[q % 4],       F.R[(q + 3) % 4], F.R[(q + 2) % 4],  F.R[(q + 1) % 4]};
}

// One fused sweep over blocks [b0, b1): copy, one launch per block (launch_q
// enqueues the kernel of block [lo, hi) at position q), flush.  Profiling
// samples the per-block launches evenly.
template <class LaunchQ>
static void enqueue_fused(pct_plan &pl, const FusedBufs &F, int64_t b0, int64_t b1, int64_t block, int64_t n,
                          hipStream_t s, bool record_events, int64_t every, LaunchQ launch_q, int full = 0)
{
    hipLaunchKernelGGL(k_sweep_begin, dim3(F.copy_grid), dim3(256), 0, s, F.X[0], F.X[1], F.R[0], F.nv);
    int64_t q = 0;
    for (int64_t t = b0; t < b1; ++t, ++q) {
        const int64_t lo = t * block;
        const int64_t hi = std::min<int64_t>(n, lo + block);
        const bool sample = record_events && (q % every == 0) && pl.prof_used[0] < kProfSamples;
        if (sample) (void)hipEventRecord(prof_event(pl, 0, 2 * pl.prof_used[0]), s);
        launch_q(s, q, lo, hi, fused_step(F, q));
        if (sample) {
            (void)hipEventRecord(prof_event(pl, 0, 2 * pl.prof_used[0] + 1), s);
            pl.prof_used[0]++;
        }
    }
    if (q > 0) {
        const int64_t last = q - 1;
        hipLaunchKernelGGL(k_sweep_end, dim3(F.copy_grid), dim3(256), 0, s, F.X[0], F.X[q % 2], F.PK[last % 3],
                           F.PK[(last + 2) % 3], F.R[last % 4], F.R[(last + 3) % 4], F.nv, full);
    }
}

// Runs n_iter sweeps: directly on the stream, or captured once into a HIP
// graph (cached on the plan for an identical launch key) and replayed.
template <class Sweep>
static int run_sweeps(pct_plan &pl, const std::vector<uint64_t> &key, bool use_graph, int n_iter, bool prof,
                      hipStream_t s, Sweep sweep)
{
    if (!use_graph) {
        for (int it = 0; it < n_iter; ++it) sweep(s, prof && it == n_iter - 1);
        return hipGetLastError();
    }
    if (!pl.graph_exec || pl.graph_key != key) {
        // recorded on a private stream (the caller's stream may be the null
        // stream, which cannot be captured); launched on the caller's stream
        if (pl.graph_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(pl.graph_exec));
        pl.graph_exec = nullptr;
        pl.graph_key.clear();
        if (!pl.capture_stream) {
            hipStream_t cs = nullptr;
            hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
            if (e != hipSuccess) return e;
            pl.capture_stream = cs;
        }
        hipStream_t cs = static_cast<hipStream_t>(pl.capture_stream);
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        sweep(cs, false);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        if (e != hipSuccess) return e;
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        pl.graph_exec = exec;
        pl.graph_key = key;
    }
    for (int it = 0; it < n_iter; ++it) {
        hipError_t e = hipGraphLaunch(static_cast<hipGraphExec_t>(pl.graph_exec), s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static inline uint64_t bits_of(double v)
{
    uint64_t u;
    std::memcpy(&u, &v, sizeof(u));
    return u;
}

template <typename T, int CHORD, bool HULL>
static int drop_loop(pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, T *x,
                     const pct_drop_opts &o, void *ws, size_t ws_bytes, hipStream_t s)
{
    const bool prof = (o.flags & PCT_DROP_PROFILE) != 0;
    if (prof) {
        hipError_t e = prof_prepare(pl);
        if (e != hipSuccess) return e;
    }
    const int lanes = choose_lanes(pl, o.lanes);
    const int64_t nblk = o.block_end - o.block_begin;
    const int64_t every = std::max<int64_t>(1, (nblk + kProfSamples - 1) / kProfSamples);
    Layout L = layout_for(pl.nvox, pl.K, o.dtype);
    const PathSrc src = path_src(pl, wsb(ws) + L.table);
    unsigned *status = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr) + kHdrStatus;
    int *hdr = reinterpret_cast<int *>(wsb(ws) + L.hdr);
    void *acc = wsb(ws) + L.acc;
    int32_t *cnt = reinterpret_cast<int32_t *>(wsb(ws) + L.cnt);
    GridDev g = grid_dev(pl.grid);
    const unsigned commit_grid = unsigned(std::min<int64_t>(4096, (pl.nvox + kWG - 1) / kWG));
    const bool cancellable = (o.flags & PCT_DROP_CANCELLABLE) != 0;
    const GateDev gate = gate_dev(ws, L, cancellable);
    // FP64 deterministic mode: integer block sums in the first two accumulators
    const bool det = sizeof(T) == 8 && (o.flags & PCT_DROP_DETERMINISTIC) != 0;
    long long *acc_lo = det ? reinterpret_cast<long long *>(wsb(ws) + L.acc + L.acc_stride) : nullptr;

    // Separate schedule: re-arm the range words, then block kernel + commit
    // per block.
    auto enqueue_sweep = [&](hipStream_t s, bool record_events) {
        hipLaunchKernelGGL(k_reset_ranges, dim3(1), dim3(64), 0, s, hdr);
        int64_t seq = 0;
        for (int64_t t = o.block_begin; t < o.block_end; ++t, ++seq) {
            int64_t lo = t * o.block;
            int64_t hi = std::min<int64_t>(n, lo + o.block);
            int *r_this = hdr + (seq % 2 == 0 ? kHdrRange0 : kHdrRange1);
            int *r_next = hdr + (seq % 2 == 0 ? kHdrRange1 : kHdrRange0);
            const bool sample = record_events && (seq % every == 0) && pl.prof_used[0] < kProfSamples;
            if (sample) (void)hipEventRecord(prof_event(pl, 0, 2 * pl.prof_used[0]), s);
            launch_block<T, CHORD, HULL>(lanes, s, p, b, x, acc, cnt, r_this, src, g, lo, hi, o.lambda, status,
                                         acc_lo, gate.halt);
            if (sample) {
                (void)hipEventRecord(prof_event(pl, 0, 2 * pl.prof_used[0] + 1), s);
                pl.prof_used[0]++;
                (void)hipEventRecord(prof_event(pl, 1, 2 * pl.prof_used[1]), s);
            }
            hipLaunchKernelGGL(k_drop_commit<T>, dim3(commit_grid), dim3(kWG), 0, s, x, acc, cnt, r_this, r_next,
                               acc_lo, gate);
            if (sample) {
                (void)hipEventRecord(prof_event(pl, 1, 2 * pl.prof_used[1] + 1), s);
                pl.prof_used[1]++;
            }
        }
    };
    // binned schedule (FP32 default): the workspace holds the slab bins of a
    // block and a slab's window fits the LDS budget
    const int nslab = std::max(pl.grid.nx, pl.grid.ny);
    const int win_words = sizeof(T) == 4 ? slab_window_words() : 0;
    const bool binned = sizeof(T) == 4 && lanes > 1 && !(o.flags & (PCT_DROP_SEPARATE_COMMIT | PCT_DROP_FUSED_COMMIT)) &&
                        nslab <= win_words && o.block <= kBinMaxRows && pl.nvox < (int64_t(1) << 30) &&
                        ws_bytes >= L.total + 2 * slot_bytes(o.block) + bin_bytes(o.block, nslab);
    const bool comp = binned && !(o.flags & PCT_DROP_NO_COMPENSATION);
    const bool fused = sizeof(T) == 4 && lanes > 1 && !(o.flags & PCT_DROP_SEPARATE_COMMIT) && !binned && !cancellable;
    // tracing ahead doubles the workgroups of a launch; with blocks above
    // kPipeMaxBlock protons the plain fused schedule is the faster one
    // (measured: 3200-proton blocks 165 vs 169 ms per sweep traced ahead, 6400-proton
    // blocks 953 vs 871 ms on the 256 x 256 x 64 scan)
    const bool pipe = fused && lanes == 64 && !(o.flags & PCT_DROP_NO_TRACE_AHEAD) && o.block <= kPipeMaxBlock &&
                      ws_bytes >= L.total + 2 * slot_bytes(o.block);
    auto sweep = [&](hipStream_t s, bool record_events) {
        if constexpr (sizeof(T) == 4) {
            if (binned) {
                BinsDev bins;
                const int64_t cap = bin_rows(o.block);
                char *bbase = wsb(ws) + L.total + 2 * slot_bytes(o.block);
                const size_t nrow = size_t(nslab) * size_t(cap);
                bins.w = reinterpret_cast<unsigned long long *>(bbase);
                bins.j1 = reinterpret_cast<unsigned *>(bbase + nrow * kBinCap * 8);
                bins.j0 = reinterpret_cast<unsigned *>(bbase + nrow * (kBinCap * 8 + (kBinCap - 1) * 4));
                bins.rowmax = reinterpret_cast<float *>(bbase + nrow * (kBinCap * 8 + (kBinCap - 1) * 4 + 2 * 4));
                bins.cap = int(cap);
                bins.nslab = nslab;
                const size_t ncnt = 2 * nrow;
                int *ovf_flag = hdr + kHdrOvf;
                unsigned long long *ovf = static_cast<unsigned long long *>(acc);
                const int zc = std::min(pl.grid.nz, win_words / nslab);
                const int nzc = (pl.grid.nz + zc - 1) / zc;
                const size_t win_lds = size_t(nslab) * size_t(zc) * sizeof(unsigned long long);
                float *xlo = reinterpret_cast<float *>(wsb(ws) + L.lo);
                hipLaunchKernelGGL(k_bins_begin, dim3(unsigned(std::min<size_t>(1024, (ncnt / 4 + 255) / 256 + 1))),
                                   dim3(256), 0, s, bins.j0, ncnt, ovf_flag);
                int64_t seq = 0;
                for (int64_t t = o.block_begin; t < o.block_end; ++t, ++seq) {
                    const int64_t lo = t * o.block;
                    const int64_t hi = std::min<int64_t>(n, lo + o.block);
                    const int par = int(seq & 1);
                    // sampled blocks: both kernels timed by their own launch events
                    const bool sample = record_events && (seq % every == 0) && pl.prof_used[0] < kProfSamples;
                    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
                    if (sample) {
                        e[0] = prof_event(pl, 0, 2 * pl.prof_used[0]);
                        e[1] = prof_event(pl, 0, 2 * pl.prof_used[0] + 1);
                        e[2] = prof_event(pl, 1, 2 * pl.prof_used[1]);
                        e[3] = prof_event(pl, 1, 2 * pl.prof_used[1] + 1);
                        pl.prof_used[0]++;
                        pl.prof_used[1]++;
                    }
                    launch_bin<CHORD, HULL>(lanes, s, p, b, reinterpret_cast<const float *>(x), bins, par, ovf,
                                            ovf_flag + par, src, g, lo, hi, o.lambda, status, gate.halt, e[0], e[1]);
                    if (sample)
                        hipExtLaunchKernelGGL(k_slab_commit, dim3(unsigned(nslab * nzc)), dim3(kSlabWG),
                                              uint32_t(win_lds), s, e[2], e[3], 0u, p, lo, int(hi - lo), bins, par,
                                              ovf, ovf_flag, reinterpret_cast<float *>(x), xlo, g, zc, nzc,
                                              comp ? 1 : 0, status, gate);
                    else
                        hipLaunchKernelGGL(k_slab_commit, dim3(unsigned(nslab * nzc)), dim3(kSlabWG), win_lds, s, p,
                                           lo, int(hi - lo), bins, par, ovf, ovf_flag, reinterpret_cast<float *>(x),
                                           xlo, g, zc, nzc, comp ? 1 : 0, status, gate);
                }
                return;
            }
            if (pipe) {
                const FusedBufs F = fused_bufs(pl, ws, x);
                SlotDev slot[2] = {slot_at(wsb(ws) + L.total, o.block),
                                   slot_at(wsb(ws) + L.total + slot_bytes(o.block), o.block)};
                const size_t lds = 3 * size_t(src.nvmax) * sizeof(double) + stash_bytes<float>();
                auto block_range = [&](int64_t t, int64_t &a, int64_t &e) {
                    a = e = 0;
                    if (t < o.block_end) {
                        a = t * o.block;
                        e = std::min<int64_t>(n, a + o.block);
                    }
                };
                enqueue_fused(pl, F, o.block_begin, o.block_end, o.block, n, s, record_events, every,
                              [&](hipStream_t s, int64_t q, int64_t lo, int64_t hi, const FusedStep &f) {
                                  int64_t wlo, whi;
                                  if (q == 0) {  // prologue: trace the first block
                                      block_range(o.block_begin, wlo, whi);
                                      hipLaunchKernelGGL((k_drop_pipe<CHORD, HULL>), dim3(unsigned(8 * ((whi - wlo + 7) / 8))),
                                                         dim3(64),
                                                         lds, s, p, b, f.base, f.next, f.pk_prev, f.pk_cur,
                                                         f.pk_old, f.r_cur, f.r_prev, f.r_old, f.r_reset, slot[1],
                                                         slot[0], src, g, int64_t(0), int64_t(0), wlo, whi, 0,
                                                         o.lambda, status, F.nv, 1);
                                  }
                                  // the commit scans the whole volume (full = 1): a block's
                                  // touched index range spans nearly all of it in these
                                  // angle-major scans, and skipping the range words saves the
                                  // DROP step their same-address atomics (165 -> 159 ms per
                                  // sweep on the 10^7-proton 200x200x32 scan)
                                  block_range(o.block_begin + q + 1, wlo, whi);
                                  const int64_t n_d = hi - lo;
                                  const unsigned grid =
                                      unsigned(kCommitWG + 8 * ((whi - wlo + 7) / 8) + 8 * ((n_d + 7) / 8));
                                  hipLaunchKernelGGL((k_drop_pipe<CHORD, HULL>), dim3(grid), dim3(64), lds, s, p, b, f.base,
                                                     f.next, f.pk_prev, f.pk_cur, f.pk_old, f.r_cur, f.r_prev,
                                                     f.r_old, f.r_reset, slot[q % 2], slot[(q + 1) % 2], src,
                                                     g, lo, hi, wlo, whi, kCommitWG, o.lambda, status, F.nv, 1);
                              }, 1);
                return;
            }
            if (fused) {
                const FusedBufs F = fused_bufs(pl, ws, x);
                enqueue_fused(pl, F, o.block_begin, o.block_end, o.block, n, s, record_events, every,
                              [&](hipStream_t s, int64_t, int64_t lo, int64_t hi, const FusedStep &f) {
                                  launch_fused<CHORD, HULL>(lanes, s, p, b, f.base, f.next, f.pk_prev, f.pk_cur, f.pk_old,
                                                      f.r_cur, f.r_prev, f.r_old, f.r_reset, src, g, lo, hi,
                                                      o.lambda, status, F.nv, 1);   // whole-volume commit
                              }, 1);
                return;
            }
        }
        enqueue_sweep(s, record_events);
    };
    const bool use_graph = !(o.flags & PCT_DROP_NO_GRAPH) && !prof;
    std::vector<uint64_t> key = {
        reinterpret_cast<uint64_t>(p.t_in),   reinterpret_cast<uint64_t>(p.v_in),
        reinterpret_cast<uint64_t>(p.th_in),  reinterpret_cast<uint64_t>(p.ph_in),
        reinterpret_cast<uint64_t>(p.t_out),  reinterpret_cast<uint64_t>(p.v_out),
        reinterpret_cast<uint64_t>(p.th_out), reinterpret_cast<uint64_t>(p.ph_out),
        reinterpret_cast<uint64_t>(p.gantry), reinterpret_cast<uint64_t>(b),
        reinterpret_cast<uint64_t>(x),        reinterpret_cast<uint64_t>(ws),
        uint64_t(n), uint64_t(o.block), uint64_t(o.block_begin), uint64_t(o.block_end),
        uint64_t(o.dtype), uint64_t(CHORD), uint64_t(lanes),
        uint64_t(fused) + 2 * uint64_t(pipe) + 4 * uint64_t(binned) + 8 * uint64_t(comp) + 16 * uint64_t(cancellable) +
            32 * uint64_t(det),
        bits_of(o.lambda),
        0};
    if (cancellable) hipLaunchKernelGGL(k_gate_begin, dim3(1), dim3(64), 0, s, gate);
    if (comp) {
        // the compensation words start at zero in every call (outside the graph)
        hipLaunchKernelGGL(k_zero_f32, dim3(unsigned(std::min<int64_t>(2048, (pl.nvox + 255) / 256))), dim3(256), 0, s,
                           reinterpret_cast<float *>(wsb(ws) + L.lo), pl.nvox);
    }
    return run_sweeps(pl, key, use_graph, o.n_iter, prof, s, sweep);
}

template <typename T>
static int drop_dispatch_chord(pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, T *x,
                               const pct_drop_opts &o, void *ws, size_t wsb_, hipStream_t s)
{
    auto go = [&](auto hull) -> int {
        constexpr bool H = decltype(hull)::value;
        switch (o.chord) {
        case PCT_CHORD_F32: return drop_loop<T, PCT_CHORD_F32, H>(pl, p, n, b, x, o, ws, wsb_, s);
        case PCT_CHORD_F16: return drop_loop<T, PCT_CHORD_F16, H>(pl, p, n, b, x, o, ws, wsb_, s);
        case PCT_CHORD_BF16: return drop_loop<T, PCT_CHORD_BF16, H>(pl, p, n, b, x, o, ws, wsb_, s);
        default: return drop_loop<T, PCT_CHORD_F64, H>(pl, p, n, b, x, o, ws, wsb_, s);
        }
    };
    return pl.hull ? go(std::true_type{}) : go(std::false_type{});
}

int launch_drop(pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, void *x, const pct_drop_opts &o,
                void *ws, size_t ws_bytes, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (o.dtype == PCT_F64)
        return drop_dispatch_chord<double>(pl, p, n, b, static_cast<double *>(x), o, ws, ws_bytes, s);
    return drop_dispatch_chord<float>(pl, p, n, b, static_cast<float *>(x), o, ws, ws_bytes, s);
}

int launch_span_histogram(const pct_plan &pl, const ProtonsDev &p, int64_t n, int64_t *hist, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const GridDev g = grid_dev(pl.grid);
    const unsigned grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(2048, (n + kSelWG - 1) / kSelWG)));
    hipLaunchKernelGGL(k_span_histogram, dim3(grid), dim3(kSelWG), size_t(pl.grid.nz) * sizeof(unsigned), s, p, n, g,
                       reinterpret_cast<unsigned long long *>(hist));
    return hipGetLastError();
}

int launch_order_blocks(const pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, int64_t block,
                        const ProtonsBufDev &out, float *b_out, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    int p2 = 2;
    while (p2 < block && p2 < n) p2 <<= 1;
    const int64_t nb = (n + block - 1) / block;
    hipLaunchKernelGGL(k_order_blocks, dim3(unsigned(nb)), dim3(kSelWG), size_t(p2) * sizeof(unsigned long long), s, p,
                       b, n, block, p2, grid_dev(pl.grid), out, b_out);
    return hipGetLastError();
}

int copy_device(void *dst, const void *src, size_t bytes, void *stream)
{
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
}

int launch_region_select(const pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, int z_lo, int z_hi,
                         const ProtonsBufDev &out, int64_t capacity, float *b_out, int64_t *count, void *ws,
                         void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    long long *partial = reinterpret_cast<long long *>(wsb(ws) + L.partial);
    const GridDev g = grid_dev(pl.grid);
    const int64_t G = std::max<int64_t>(1, std::min<int64_t>(kMaxPartials, (n + kSelWG - 1) / kSelWG));
    int64_t chunk = (n + G - 1) / G;
    chunk = std::max<int64_t>(kSelWG, (chunk + kSelWG - 1) / kSelWG * kSelWG);
    hipLaunchKernelGGL(k_region_count, dim3(unsigned(G)), dim3(kSelWG), 0, s, p, n, chunk, g, z_lo, z_hi, partial);
    hipLaunchKernelGGL(k_region_scan, dim3(1), dim3(kSelWG), 0, s, partial, int(G), count);
    hipLaunchKernelGGL(k_region_scatter, dim3(unsigned(G)), dim3(kSelWG), 0, s, p, b, n, chunk, g, z_lo, z_hi,
                       partial, out, capacity, b_out);
    return hipGetLastError();
}

__global__ void k_zero_i64(long long *p, int64_t n)
{
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

int launch_rows_count(const pct_plan &pl, const ProtonsDev &p, int64_t n, int64_t *offsets, void *ws, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    const PathSrc src = path_src(pl, wsb(ws) + L.table);
    unsigned *status = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr) + kHdrStatus;
    long long *partial = reinterpret_cast<long long *>(wsb(ws) + L.partial);
    long long *off = reinterpret_cast<long long *>(offsets);
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, s, off, int64_t(1));
    if (n > 0) {
if (src.hull)
                    hipLaunchKernelGGL(k_row_lengths<true>, dim3(grid_for(n)), dim3(kWG), 0, s, p, n, off + 1, src,
                           grid_dev(pl.grid), status);
        else
                    hipLaunchKernelGGL(k_row_lengths<false>, dim3(grid_for(n)), dim3(kWG), 0, s, p, n, off + 1, src,
                           grid_dev(pl.grid), status);
        const int64_t G = std::max<int64_t>(1, std::min<int64_t>(kMaxPartials, (n + kSelWG - 1) / kSelWG));
        int64_t chunk = (n + G - 1) / G;
        chunk = std::max<int64_t>(kSelWG, (chunk + kSelWG - 1) / kSelWG * kSelWG);
        hipLaunchKernelGGL(k_chunk_sums, dim3(unsigned(G)), dim3(kSelWG), 0, s, off + 1, n, chunk, partial);
        hipLaunchKernelGGL(k_region_scan, dim3(1), dim3(kSelWG), 0, s, partial, int(G),
                           static_cast<int64_t *>(nullptr));
        hipLaunchKernelGGL(k_chunk_scan, dim3(unsigned(G)), dim3(kSelWG), 0, s, off + 1, n, chunk, partial);
    }
    return hipGetLastError();
}

int launch_rows_build(const pct_plan &pl, const ProtonsDev &p, int64_t n, int chord_type, const int64_t *offsets,
                      int32_t *vox, void *chord, double *n2, void *ws, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    const PathSrc src = path_src(pl, wsb(ws) + L.table);
    unsigned *status = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr) + kHdrStatus;
    const long long *off = reinterpret_cast<const long long *>(offsets);
    const GridDev g = grid_dev(pl.grid);
    switch (chord_type) {
    case PCT_CHORD_F16:
        if (src.hull)
            hipLaunchKernelGGL((k_rows_build<PCT_CHORD_F16, true>), dim3(grid_for(n)), dim3(kWG), 0, s, p, n, off, vox,
                           static_cast<unsigned short *>(chord), n2, src, g, status);
        else
            hipLaunchKernelGGL((k_rows_build<PCT_CHORD_F16, false>), dim3(grid_for(n)), dim3(kWG), 0, s, p, n, off, vox,
                           static_cast<unsigned short *>(chord), n2, src, g, status);
        break;
    case PCT_CHORD_BF16:
        if (src.hull)
            hipLaunchKernelGGL((k_rows_build<PCT_CHORD_BF16, true>), dim3(grid_for(n)), dim3(kWG), 0, s, p, n, off, vox,
                           static_cast<unsigned short *>(chord), n2, src, g, status);
        else
            hipLaunchKernelGGL((k_rows_build<PCT_CHORD_BF16, false>), dim3(grid_for(n)), dim3(kWG), 0, s, p, n, off, vox,
                           static_cast<unsigned short *>(chord), n2, src, g, status);
        break;
    default:
        if (src.hull)
            hipLaunchKernelGGL((k_rows_build<PCT_CHORD_F32, true>), dim3(grid_for(n)), dim3(kWG), 0, s, p, n, off, vox,
                           static_cast<float *>(chord), n2, src, g, status);
        else
            hipLaunchKernelGGL((k_rows_build<PCT_CHORD_F32, false>), dim3(grid_for(n)), dim3(kWG), 0, s, p, n, off, vox,
                           static_cast<float *>(chord), n2, src, g, status);
    }
    return hipGetLastError();
}

template <int CT>
static void launch_rows_fused(int lanes, hipStream_t s, const RowsDev &rows, const float *b, const FusedStep &f,
                              int64_t lo, int64_t hi, double lambda, unsigned *status, int nvox)
{
    const int64_t n = hi - lo;
    switch (lanes) {
#define PCT_LAUNCH_ROWS(LPR)                                                                                     \
    case LPR: {                                                                                                  \
        const unsigned grid = unsigned(kCommitWG + (n + (64 / LPR) - 1) / (64 / LPR));                        \
        hipLaunchKernelGGL((k_drop_rows_fused<CT, LPR>), dim3(grid), dim3(64), 0, s, rows, b, f.base, f.next,     \
                           f.pk_prev, f.pk_cur, f.pk_old, f.r_cur, f.r_prev, f.r_old, f.r_reset, lo, hi, lambda,  \
                           status, nvox);                                                                        \
        break;                                                                                                   \
    }
        PCT_LAUNCH_ROWS(16)
        PCT_LAUNCH_ROWS(32)
        PCT_LAUNCH_ROWS(64)
#undef PCT_LAUNCH_ROWS
    default: break;
    }
}

int launch_drop_rows(pct_plan &pl, const pct_rows &rows, const float *b, float *x, const pct_drop_opts &o, void *ws,
                     void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool prof = (o.flags & PCT_DROP_PROFILE) != 0;
    if (prof) {
        hipError_t e = prof_prepare(pl);
        if (e != hipSuccess) return e;
    }
    const int lanes = o.lanes == 0 ? 64 : o.lanes;
    const int64_t nblk = o.block_end - o.block_begin;
    const int64_t every = std::max<int64_t>(1, (nblk + kProfSamples - 1) / kProfSamples);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    unsigned *status = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr) + kHdrStatus;
    const RowsDev rd{reinterpret_cast<const long long *>(rows.offsets), rows.vox, rows.chord, rows.n2};
    const int64_t n = rows.n;
    auto sweep = [&](hipStream_t s, bool record_events) {
        const FusedBufs F = fused_bufs(pl, ws, x);
        enqueue_fused(pl, F, o.block_begin, o.block_end, o.block, n, s, record_events, every,
                      [&](hipStream_t s, int64_t, int64_t lo, int64_t hi, const FusedStep &f) {
                          switch (rows.chord_type) {
                          case PCT_CHORD_F16:
                              launch_rows_fused<PCT_CHORD_F16>(lanes, s, rd, b, f, lo, hi, o.lambda, status, F.nv);
                              break;
                          case PCT_CHORD_BF16:
                              launch_rows_fused<PCT_CHORD_BF16>(lanes, s, rd, b, f, lo, hi, o.lambda, status, F.nv);
                              break;
                          default:
                              launch_rows_fused<PCT_CHORD_F32>(lanes, s, rd, b, f, lo, hi, o.lambda, status, F.nv);
                          }
                      });
    };
    const bool use_graph = !(o.flags & PCT_DROP_NO_GRAPH) && !prof;
    std::vector<uint64_t> key = {reinterpret_cast<uint64_t>(rows.offsets), reinterpret_cast<uint64_t>(rows.vox),
                                 reinterpret_cast<uint64_t>(rows.chord),   reinterpret_cast<uint64_t>(rows.n2),
                                 reinterpret_cast<uint64_t>(b),            reinterpret_cast<uint64_t>(x),
                                 reinterpret_cast<uint64_t>(ws),           uint64_t(n),
                                 uint64_t(o.block),                        uint64_t(o.block_begin),
                                 uint64_t(o.block_end),                    uint64_t(rows.chord_type),
                                 uint64_t(lanes),                          bits_of(o.lambda),
                                 1};
    return run_sweeps(pl, key, use_graph, o.n_iter, prof, s, sweep);
}

static int tv_into(const pct_plan &pl, const void *x, int dtype, double eps, double *value_dev, void *grad,
                   double *partial, hipStream_t s)
{
    int nblk = int(std::min<int64_t>(kMaxPartials, (pl.nvox + kWG - 1) / kWG));
    if (dtype == PCT_F64)
        hipLaunchKernelGGL(k_tv<double>, dim3(nblk), dim3(kWG), 0, s, static_cast<const double *>(x),
                           grid_dev(pl.grid), eps, static_cast<double *>(grad), partial, pl.nvox);
    else
        hipLaunchKernelGGL(k_tv<float>, dim3(nblk), dim3(kWG), 0, s, static_cast<const float *>(x),
                           grid_dev(pl.grid), eps, static_cast<float *>(grad), partial, pl.nvox);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kWG), 0, s, partial, nblk, value_dev);
    return hipGetLastError();
}

int launch_tv(const pct_plan &pl, const void *x, int dtype, double eps, double *value_dev, void *grad, void *ws,
              void *stream)
{
    const Layout L = layout_for(pl.nvox, pl.K, dtype);
    return tv_into(pl, x, dtype, eps, value_dev, grad, reinterpret_cast<double *>(wsb(ws) + L.partial),
                   static_cast<hipStream_t>(stream));
}

// TV without a workspace: the per-workgroup partial sums (at most
// kMaxPartials doubles, 32 KB) live in this file-scope device array, one copy
// per GPU, held until the process ends.  Host code never passes the array's
// name to a kernel: its device address is looked up once per device (with
// that device current) and kept.  Calls on one GPU share the array, so calls
// that overlap on one GPU race; every partial a call reads it has written
// first, so nothing needs clearing.
static __device__ __align__(256) double scratch[kMaxPartials];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch[kMaxScratchDevices];

static hipError_t scratch_address(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

int launch_tv_static(const pct_plan &pl, const void *x, int dtype, double eps, double *value_dev, void *grad,
                     void *stream)
{
    double *partial = nullptr;
    const hipError_t e = scratch_address(&partial);
    if (e != hipSuccess) return e;
    return tv_into(pl, x, dtype, eps, value_dev, grad, partial, static_cast<hipStream_t>(stream));
}

}  // namespace pct
