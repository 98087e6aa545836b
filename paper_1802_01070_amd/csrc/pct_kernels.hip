// HIP kernels of the reconstruction path for gfx950 and their launchers.
//
//   k_trace        ordered emission list of each proton's path (debug/parity)
//   k_forward      y = A x, ||a_i||^2   (one lane per proton, gathers)
//   k_backproject  g += A^T r           (one lane per proton, atomics)
//   k_drop_rows    DROP block: walk -> a_i.x, ||a_i||^2 -> rho_i -> re-walk and
//                  scatter rho_i a_ij into the block accumulator and the
//                  per-voxel row count, first touch appends to a touched list
//   k_drop_commit  x_j += acc_j / s_j over the touched list, reset
//   k_tv           smoothed total variation value and gradient
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pct_internal.h"
#include "pct_path.hpp"

namespace pct {

constexpr int kWG = 256;

__device__ __forceinline__ void raise_status(unsigned *status, unsigned bit)
{
    atomicOr(status, bit);
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

__global__ void __launch_bounds__(kWG) k_trace(ProtonsDev p, int64_t first, int64_t count, int32_t max_nnz,
                                               int32_t *vox, double *chord, int32_t *nnz,
                                               const double *__restrict__ tab, int K, GridDev g, unsigned *status)
{
    int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= count) return;
    Rec r = load_rec(p, first + q);
    TraceSink ts{vox + q * max_nnz, chord + q * max_nnz, max_nnz, 0};
    if (rec_finite(r)) {
        Merge<TraceSink, PCT_CHORD_F64> m(ts, g);
        walk_path(r, tab, K, g, m);
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
template <typename T>
struct DotSink {
    const T *__restrict__ x;
    Reentry re;
    double dot, n2;
    __device__ __forceinline__ void segment(double dx, double dy) { re.segment(dx, dy); }
    __device__ __forceinline__ void final(int j, int ix, int iy, int iz, double c)
    {
        bool first;
        double aprev = re.visit(j, ix, iy, iz, c, first);
        dot += c * double(x[j]);
        n2 += c * (2.0 * aprev + c);
    }
};

template <typename T>
__global__ void __launch_bounds__(kWG) k_forward(ProtonsDev p, int64_t n, const T *__restrict__ x, T *y, T *nrm2,
                                                 const double *__restrict__ tab, int K, GridDev g, unsigned *status)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Rec r = load_rec(p, i);
    DotSink<T> s;
    s.x = x;
    s.dot = 0.0;
    s.n2 = 0.0;
    s.re.init(r);
    if (rec_finite(r)) {
        Merge<DotSink<T>, PCT_CHORD_F64> m(s, g);
        walk_path(r, tab, K, g, m);
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
template <typename T>
struct ScatterSink {
    T *g;
    double r;
    __device__ __forceinline__ void segment(double, double) {}
    __device__ __forceinline__ void final(int j, int, int, int, double c) { atomicAdd(g + j, T(r * c)); }
};

template <typename T>
__global__ void __launch_bounds__(kWG) k_backproject(ProtonsDev p, int64_t n, const T *__restrict__ rv, T *gout,
                                                     const double *__restrict__ tab, int K, GridDev g,
                                                     unsigned *status)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ri = double(rv[i]);
    if (ri == 0.0) return;
    Rec r = load_rec(p, i);
    if (!rec_finite(r) || !isfinite(ri)) {
        raise_status(status, PCT_DEV_NONFINITE);
        return;
    }
    ScatterSink<T> s{gout, ri};
    Merge<ScatterSink<T>, PCT_CHORD_F64> m(s, g);
    walk_path(r, tab, K, g, m);
    m.finish();
}

// ---------------------------------------------------------------------------
// DROP
// ---------------------------------------------------------------------------
template <typename T>
struct DropScatterSink {
    T *acc;
    int32_t *cnt;
    int32_t *touched;
    unsigned *ntouched;
    Reentry re;
    double rho;
    __device__ __forceinline__ void segment(double dx, double dy) { re.segment(dx, dy); }
    __device__ __forceinline__ void final(int j, int ix, int iy, int iz, double c)
    {
        bool first;
        re.visit(j, ix, iy, iz, c, first);
        atomicAdd(acc + j, T(rho * c));
        if (first) {
            int old = atomicAdd(cnt + j, 1);
            if (old == 0) touched[atomicAdd(ntouched, 1u)] = j;
        }
    }
};

template <typename T, int CHORD>
__global__ void __launch_bounds__(kWG) k_drop_rows(ProtonsDev p, const float *__restrict__ b,
                                                   const T *__restrict__ x, T *acc, int32_t *cnt, int32_t *touched,
                                                   unsigned *ntouched, const double *__restrict__ tab, int K,
                                                   GridDev g, int64_t lo, int64_t hi, double lambda,
                                                   unsigned *status)
{
    int64_t i = lo + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= hi) return;
    Rec r = load_rec(p, i);
    double bi = double(b[i]);
    if (!rec_finite(r) || !isfinite(bi)) {
        raise_status(status, PCT_DEV_NONFINITE);
        return;
    }
    DotSink<T> s;
    s.x = x;
    s.dot = 0.0;
    s.n2 = 0.0;
    s.re.init(r);
    {
        Merge<DotSink<T>, CHORD> m(s, g);
        walk_path(r, tab, K, g, m);
        m.finish();
    }
    if (s.re.unsafe) raise_status(status, PCT_DEV_REENTRY);
    if (!(s.n2 > 0.0)) return;
    DropScatterSink<T> sc;
    sc.acc = acc;
    sc.cnt = cnt;
    sc.touched = touched;
    sc.ntouched = ntouched;
    sc.rho = lambda * (bi - s.dot) / s.n2;
    sc.re.init(r);
    Merge<DropScatterSink<T>, CHORD> m(sc, g);
    walk_path(r, tab, K, g, m);
    m.finish();
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_drop_commit(T *x, T *acc, int32_t *cnt, const int32_t *__restrict__ touched,
                                                     const unsigned *ntouched_this, unsigned *ntouched_next)
{
    const unsigned n = *ntouched_this;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ntouched_next = 0u;
    for (unsigned q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        int j = touched[q];
        double s = double(cnt[j]);
        x[j] = T(double(x[j]) + double(acc[j]) / s);
        acc[j] = T(0);
        cnt[j] = 0;
    }
}

__global__ void k_reset_counters(unsigned *hdr)
{
    if (threadIdx.x == 0) {
        hdr[kHdrTouched0] = 0u;
        hdr[kHdrTouched1] = 0u;
    }
}

// ---------------------------------------------------------------------------
// total variation
// ---------------------------------------------------------------------------
__device__ __forceinline__ double tv_diffs(const float *__restrict__ x, const GridDev &g, int ix, int iy, int iz,
                                           int64_t v, double eps, double &dx, double &dy, double &dz)
{
    const int64_t sy = g.n[0], sz = int64_t(g.n[0]) * g.n[1];
    double xv = x[v];
    dx = ix + 1 < g.n[0] ? double(x[v + 1]) - xv : 0.0;
    dy = iy + 1 < g.n[1] ? double(x[v + sy]) - xv : 0.0;
    dz = iz + 1 < g.n[2] ? double(x[v + sz]) - xv : 0.0;
    return sqrt(dx * dx + dy * dy + dz * dz + eps * eps);
}

__global__ void __launch_bounds__(kWG) k_tv(const float *__restrict__ x, GridDev g, double eps, float *grad,
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
            grad[v] = float(gv);
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

int launch_trace(const pct_plan &pl, const ProtonsDev &p, int64_t first, int64_t count, int32_t max_nnz,
                 int32_t *vox, double *chord, int32_t *nnz, void *ws, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    const double *tab = reinterpret_cast<const double *>(wsb(ws) + L.table);
    unsigned *status = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr) + kHdrStatus;
    hipLaunchKernelGGL(k_trace, dim3(grid_for(count)), dim3(kWG), 0, s, p, first, count, max_nnz, vox, chord, nnz,
                       tab, pl.K, grid_dev(pl.grid), status);
    return hipGetLastError();
}

int launch_forward(const pct_plan &pl, const ProtonsDev &p, int64_t n, const void *x, int dtype, void *y,
                   void *nrm2, void *ws, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    const double *tab = reinterpret_cast<const double *>(wsb(ws) + L.table);
    unsigned *status = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr) + kHdrStatus;
    GridDev g = grid_dev(pl.grid);
    if (dtype == PCT_F64)
        hipLaunchKernelGGL(k_forward<double>, dim3(grid_for(n)), dim3(kWG), 0, s, p, n,
                           static_cast<const double *>(x), static_cast<double *>(y), static_cast<double *>(nrm2),
                           tab, pl.K, g, status);
    else
        hipLaunchKernelGGL(k_forward<float>, dim3(grid_for(n)), dim3(kWG), 0, s, p, n, static_cast<const float *>(x),
                           static_cast<float *>(y), static_cast<float *>(nrm2), tab, pl.K, g, status);
    return hipGetLastError();
}

int launch_backproject(const pct_plan &pl, const ProtonsDev &p, int64_t n, const void *r, int dtype, void *gout,
                       void *ws, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    const double *tab = reinterpret_cast<const double *>(wsb(ws) + L.table);
    unsigned *status = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr) + kHdrStatus;
    GridDev g = grid_dev(pl.grid);
    if (dtype == PCT_F64)
        hipLaunchKernelGGL(k_backproject<double>, dim3(grid_for(n)), dim3(kWG), 0, s, p, n,
                           static_cast<const double *>(r), static_cast<double *>(gout), tab, pl.K, g, status);
    else
        hipLaunchKernelGGL(k_backproject<float>, dim3(grid_for(n)), dim3(kWG), 0, s, p, n,
                           static_cast<const float *>(r), static_cast<float *>(gout), tab, pl.K, g, status);
    return hipGetLastError();
}

template <typename T, int CHORD>
static int drop_loop(const pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, T *x,
                     const pct_drop_opts &o, void *ws, hipStream_t s)
{
    Layout L = layout_for(pl.nvox, pl.K, o.dtype);
    const double *tab = reinterpret_cast<const double *>(wsb(ws) + L.table);
    unsigned *hdr = reinterpret_cast<unsigned *>(wsb(ws) + L.hdr);
    T *acc = reinterpret_cast<T *>(wsb(ws) + L.acc);
    int32_t *cnt = reinterpret_cast<int32_t *>(wsb(ws) + L.cnt);
    int32_t *touched = reinterpret_cast<int32_t *>(wsb(ws) + L.touched);
    GridDev g = grid_dev(pl.grid);
    const unsigned commit_grid = unsigned(std::min<int64_t>(1024, (pl.nvox + kWG - 1) / kWG));
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, hdr);
    int64_t seq = 0;
    for (int it = 0; it < o.n_iter; ++it) {
        for (int64_t t = o.block_begin; t < o.block_end; ++t, ++seq) {
            int64_t lo = t * o.block;
            int64_t hi = std::min<int64_t>(n, lo + o.block);
            unsigned *nt_this = hdr + (seq % 2 == 0 ? kHdrTouched0 : kHdrTouched1);
            unsigned *nt_next = hdr + (seq % 2 == 0 ? kHdrTouched1 : kHdrTouched0);
            hipLaunchKernelGGL((k_drop_rows<T, CHORD>), dim3(grid_for(hi - lo)), dim3(kWG), 0, s, p, b, x, acc, cnt,
                               touched, nt_this, tab, pl.K, g, lo, hi, o.lambda, hdr + kHdrStatus);
            hipLaunchKernelGGL(k_drop_commit<T>, dim3(commit_grid), dim3(kWG), 0, s, x, acc, cnt, touched, nt_this,
                               nt_next);
        }
    }
    return hipGetLastError();
}

template <typename T>
static int drop_dispatch_chord(const pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, T *x,
                               const pct_drop_opts &o, void *ws, hipStream_t s)
{
    switch (o.chord) {
    case PCT_CHORD_F32: return drop_loop<T, PCT_CHORD_F32>(pl, p, n, b, x, o, ws, s);
    case PCT_CHORD_F16: return drop_loop<T, PCT_CHORD_F16>(pl, p, n, b, x, o, ws, s);
    case PCT_CHORD_BF16: return drop_loop<T, PCT_CHORD_BF16>(pl, p, n, b, x, o, ws, s);
    default: return drop_loop<T, PCT_CHORD_F64>(pl, p, n, b, x, o, ws, s);
    }
}

int launch_drop(const pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, void *x, const pct_drop_opts &o,
                void *ws, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (o.dtype == PCT_F64) return drop_dispatch_chord<double>(pl, p, n, b, static_cast<double *>(x), o, ws, s);
    return drop_dispatch_chord<float>(pl, p, n, b, static_cast<float *>(x), o, ws, s);
}

int launch_tv(const pct_plan &pl, const float *x, double eps, double *value_dev, float *grad, void *ws,
              void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    Layout L = layout_for(pl.nvox, pl.K, PCT_F32);
    double *partial = reinterpret_cast<double *>(wsb(ws) + L.partial);
    int nblk = int(std::min<int64_t>(kMaxPartials, (pl.nvox + kWG - 1) / kWG));
    hipLaunchKernelGGL(k_tv, dim3(nblk), dim3(kWG), 0, s, x, grid_dev(pl.grid), eps, grad, partial, pl.nvox);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kWG), 0, s, partial, nblk, value_dev);
    return hipGetLastError();
}

}  // namespace pct
