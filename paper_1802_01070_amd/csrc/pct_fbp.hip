// Filtered back-projection (FBP) image, the initial iterate of the iterative
// solve (Section I).  Textbook parallel-beam FBP slice by slice along each
// proton's straight entry-to-exit chord (Kak & Slaney, Principles of
// Computerized Tomographic Imaging, ch. 3):
//
//   k_fbp_bin_lds      one thread per proton: angle, lateral and slice bin of
//                      the chord at depth u = 0; bins of the workgroup's home
//                      angle summed in LDS, flushed once; k_fbp_bin, one
//                      64-bit fixed-point atomic for the WEPL sum and one
//                      32-bit atomic for the count per proton, when they do
//                      not fit (integer sums: the result does not depend on the
//                      order or on the kernel)
//   k_fbp_mean         one thread per bin: projection = mean WEPL (0 if empty)
//   k_fbp_filter       Ram-Lak ramp filter as a direct convolution over each
//                      (slice, angle) row: rows staged in LDS, a thread sums
//                      eight outputs of one parity over blocks of eight taps
//                      from row values held in registers
//   k_fbp_backproject  one thread per voxel: sum over the angles of the
//                      filtered row, linearly interpolated at the voxel's
//                      lateral coordinate; the angles' sines and cosines in LDS;
//                      workgroups of a slice stay on one XCD so that the slice's
//                      filtered rows are read through one L2; k_fbp_backproject_tiled,
//                      the same over 16 x 16 voxel tiles with each angle's
//                      row window staged in LDS (the default; the untiled
//                      kernel serves lateral bins much finer than the voxels)
//
// Sinograms are laid out [iz][angle][k] (a slice's rows are contiguous).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "pct_internal.h"

namespace pct {

constexpr double kFbpScale = 16777216.0;       // 2^24: WEPL fixed point of the bin sums
constexpr double kFbpInvScale = 1.0 / 16777216.0;
constexpr int kFbpWG = 256;

__global__ void __launch_bounds__(kFbpWG) k_fbp_clear(unsigned long long *sum, unsigned *cnt, int64_t nb)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nb; i += int64_t(gridDim.x) * blockDim.x) {
        sum[i] = 0ull;
        cnt[i] = 0u;
    }
}

__global__ void __launch_bounds__(kFbpWG) k_fbp_bin(ProtonsDev p, const float *__restrict__ b, int64_t n,
                                                    FbpDev f, unsigned long long *sum, unsigned *cnt)
{
    // the bin decisions follow the definition's operation order exactly (no
    // contraction into fused multiply-adds)
#pragma clang fp contract(off)
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const double t_in = p.t_in[i], t_out = p.t_out[i], v_in = p.v_in[i], v_out = p.v_out[i];
        const double phi = p.gantry[i], bi = b[i];
        const double tc = t_in + f.w * (t_out - t_in);
        const double vc = v_in + f.w * (v_out - v_in);
        if (!(isfinite(tc) && isfinite(vc) && isfinite(phi) && isfinite(bi))) continue;
        if (!(fabs(bi) < kFbpMaxWepl)) continue;
        const double fk = floor((tc - f.t0) / f.dt);
        const double fz = floor((vc - f.z0) / f.pz);
        if (!(fk >= 0.0 && fk < double(f.n_t) && fz >= 0.0 && fz < double(f.nz))) continue;
        double fa = fmod(floor(phi / f.dphi + 0.5), double(f.n_ang));
        if (fa < 0.0) fa += double(f.n_ang);
        const int64_t bin = (int64_t(fz) * f.n_ang + int64_t(fa)) * f.n_t + int64_t(fk);
        atomicAdd(sum + bin, static_cast<unsigned long long>(llrint(bi * kFbpScale)));
        atomicAdd(cnt + bin, 1u);
    }
}

// Privatised binning for angle-sorted scans (the acquisition order of a
// rotating gantry): workgroup w takes the contiguous protons [w chunk,
// (w+1) chunk); the bins of its home angle (that of its middle proton) are
// summed in LDS, one packed 64-bit word per (slice, lateral) bin -- count in
// bits 63..48, the 2^-24 mm fixed-point sum as a signed value below (|sum| <
// 2^47 and count < 2^15 for chunks of at most 8192 protons with |b| < 2^10
// mm) -- and flushed with one pair of global atomics per non-empty bin; other
// protons go straight to the global bins.  Integer sums: the result is that
// of k_fbp_bin bit for bit.
constexpr double kFbpLdsWepl = 1024.0;
constexpr int64_t kFbpMaxChunk = 8192;
// 1024 threads share the (up to 64 KB and more) LDS histogram: one or two
// workgroups fill a CU's LDS, so the workgroup is made wide to keep enough
// waves in flight over the chunk's loads and LDS atomics
constexpr int kFbpBinWG = 1024;

__global__ void __launch_bounds__(kFbpBinWG) k_fbp_bin_lds(ProtonsDev p, const float *__restrict__ b, int64_t n,
                                                        int64_t chunk, FbpDev f, unsigned long long *sum,
                                                        unsigned *cnt)
{
#pragma clang fp contract(off)
    extern __shared__ unsigned long long hist[];
    const int nzt = f.nz * f.n_t;
    const int64_t lo = int64_t(blockIdx.x) * chunk;
    const int64_t hi = min(n, lo + chunk);
    int home = -1;
    {
        const double phi = p.gantry[lo + (hi - 1 - lo) / 2];
        if (isfinite(phi)) {
            double fa = fmod(floor(phi / f.dphi + 0.5), double(f.n_ang));
            if (fa < 0.0) fa += double(f.n_ang);
            home = int(fa);
        }
    }
    for (int i = threadIdx.x; i < nzt; i += blockDim.x) hist[i] = 0ull;
    __syncthreads();
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double t_in = p.t_in[i], t_out = p.t_out[i], v_in = p.v_in[i], v_out = p.v_out[i];
        const double phi = p.gantry[i], bi = b[i];
        const double tc = t_in + f.w * (t_out - t_in);
        const double vc = v_in + f.w * (v_out - v_in);
        if (!(isfinite(tc) && isfinite(vc) && isfinite(phi) && isfinite(bi))) continue;
        if (!(fabs(bi) < kFbpMaxWepl)) continue;
        const double fk = floor((tc - f.t0) / f.dt);
        const double fz = floor((vc - f.z0) / f.pz);
        if (!(fk >= 0.0 && fk < double(f.n_t) && fz >= 0.0 && fz < double(f.nz))) continue;
        double fa = fmod(floor(phi / f.dphi + 0.5), double(f.n_ang));
        if (fa < 0.0) fa += double(f.n_ang);
        const long long qv = llrint(bi * kFbpScale);
        if (int(fa) == home && fabs(bi) < kFbpLdsWepl) {
            atomicAdd(hist + int(fz) * f.n_t + int(fk), (1ull << 48) + static_cast<unsigned long long>(qv));
        } else {
            const int64_t bin = (int64_t(fz) * f.n_ang + int64_t(fa)) * f.n_t + int64_t(fk);
            atomicAdd(sum + bin, static_cast<unsigned long long>(qv));
            atomicAdd(cnt + bin, 1u);
        }
    }
    __syncthreads();
    if (home < 0) return;
    for (int i = threadIdx.x; i < nzt; i += blockDim.x) {
        const unsigned long long wv = hist[i];
        if (!wv) continue;
        const long long sv = static_cast<long long>(wv << 16) >> 16;
        const unsigned c = unsigned((wv - static_cast<unsigned long long>(sv)) >> 48);
        const int iz = i / f.n_t, k = i - iz * f.n_t;
        const int64_t bin = (int64_t(iz) * f.n_ang + home) * f.n_t + k;
        atomicAdd(sum + bin, static_cast<unsigned long long>(sv));
        atomicAdd(cnt + bin, c);
    }
}

__global__ void __launch_bounds__(kFbpWG) k_fbp_mean(const unsigned long long *__restrict__ sum,
                                                     const unsigned *__restrict__ cnt, int64_t nb, double *proj,
                                                     int32_t *count)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nb; i += int64_t(gridDim.x) * blockDim.x) {
        const unsigned c = cnt[i];
        const double s = double(static_cast<long long>(sum[i])) * kFbpInvScale;
        proj[i] = c ? s / double(c) : 0.0;
        if (count) count[i] = int32_t(c);
    }
}

// q_k = dt sum_n p_n h(k - n) with h(0) = 1/(4 dt^2), h(m) = -1/(pi^2 m^2 dt^2)
// for odd m, 0 for even m: q_k = (p_k / 4 - sum_{odd m} p_{k-m} / (pi^2 m^2)) / dt,
// p zero outside the row.  A workgroup takes rpw rows (staged in LDS with the
// odd-tap coefficients c_p = 1/(pi^2 (2p+1)^2), padded with zero taps to a
// multiple of kFilterR); a thread computes kFilterR outputs of one parity,
// k0 + 2j, over blocks of kFilterR taps: the 2 kFilterR - 1 row values each
// side that a block needs are read once into registers, so the LDS reads per
// (output, tap) drop from two to about 4 / kFilterR.  Each output still sums
// its taps in ascending m, as the definition is written.
constexpr int kFilterR = 8;

__global__ void __launch_bounds__(kFbpWG) k_fbp_filter(const double *__restrict__ proj, double *__restrict__ q,
                                                       int64_t rows, int n_t, double dt, int rpw, int gpr)
{
    extern __shared__ double lds[];
    const int ntaps = n_t / 2;                                            // odd m = 2p + 1 < n_t
    const int ptaps = (ntaps + kFilterR - 1) / kFilterR * kFilterR;
    double *cm = lds;                  // ptaps coefficients, zero past ntaps
    double *rl = lds + ptaps;          // rpw rows of n_t
    const int64_t r0 = int64_t(blockIdx.x) * rpw;
    const int nr = int(min(int64_t(rpw), rows - r0));
    for (int p = threadIdx.x; p < ptaps; p += blockDim.x) {
        const double m = double(2 * p + 1);
        cm[p] = p < ntaps ? 1.0 / (M_PI * M_PI * m * m) : 0.0;
    }
    for (int i = threadIdx.x; i < nr * n_t; i += blockDim.x) rl[i] = proj[r0 * n_t + i];
    __syncthreads();
    const double inv_dt = 1.0 / dt;
    for (int wi = threadIdx.x; wi < nr * gpr; wi += blockDim.x) {
        const int r = wi / gpr, gi = wi - r * gpr;
        const int k0 = (gi & 1) + 2 * kFilterR * (gi >> 1);
        const double *row = rl + r * n_t;
        double acc[kFilterR];
#pragma unroll
        for (int j = 0; j < kFilterR; ++j) acc[j] = 0.0;
        for (int p0 = 0; p0 < ptaps; p0 += kFilterR) {
            // lo[d]: p_{k0 - 1 - 2 p0 + 2 (d - R + 1)}, the k - m term of output j and
            // tap p0 + pp at d = j - pp + R - 1; hi[d]: p_{k0 + 1 + 2 p0 + 2 d}, the k + m
            // term at d = j + pp
            double lo[2 * kFilterR - 1], hi[2 * kFilterR - 1];
#pragma unroll
            for (int d = 0; d < 2 * kFilterR - 1; ++d) {
                const int il = k0 - 1 - 2 * p0 + 2 * (d - (kFilterR - 1));
                const int ih = k0 + 1 + 2 * p0 + 2 * d;
                lo[d] = il >= 0 && il < n_t ? row[il] : 0.0;
                hi[d] = ih < n_t ? row[ih] : 0.0;
            }
#pragma unroll
            for (int pp = 0; pp < kFilterR; ++pp) {
                const double c = cm[p0 + pp];
#pragma unroll
                for (int j = 0; j < kFilterR; ++j) acc[j] += c * (lo[j - pp + kFilterR - 1] + hi[j + pp]);
            }
        }
#pragma unroll
        for (int j = 0; j < kFilterR; ++j) {
            const int k = k0 + 2 * j;
            if (k < n_t) q[(r0 + r) * n_t + k] = (0.25 * row[k] - acc[j]) * inv_dt;
        }
    }
}

// x(voxel) = (pi / n_ang) sum_a q_{iz,a}(t), t = -x sin(phi_a) + y cos(phi_a),
// linear interpolation between bin centres t0 + (k + 1/2) dt, zero beyond the
// outer bins.  Grid: 8 * ceil(nz / 8) * tiles workgroups; workgroup L runs on
// XCD L % 8 and takes slice (L % 8) + 8 * ((L / 8) / tiles), tile (L / 8) % tiles.
template <typename T>
__global__ void __launch_bounds__(kFbpWG) k_fbp_backproject(const double *__restrict__ q, T *__restrict__ x,
                                                            FbpDev f, GridDev g, int tiles)
{
    extern __shared__ double lds[];
    double *cs = lds;            // cos(phi_a)
    double *sn = lds + f.n_ang;  // sin(phi_a)
    const int L = blockIdx.x;
    const int xcd = L % 8, j = L / 8;
    const int iz = xcd + 8 * (j / tiles);
    const int tile = j % tiles;
    if (iz >= g.n[2]) return;   // whole workgroup: no barrier below is skipped by part of it
    for (int a = threadIdx.x; a < f.n_ang; a += blockDim.x) sincos(double(a) * f.dphi, &sn[a], &cs[a]);
    __syncthreads();
    const int64_t plane = int64_t(g.n[0]) * g.n[1];
    const int64_t v = int64_t(tile) * blockDim.x + threadIdx.x;
    if (v >= plane) return;
    const int ix = int(v % g.n[0]), iy = int(v / g.n[0]);
    const double xc = g.lo[0] + (ix + 0.5) * g.pitch[0];
    const double yc = g.lo[1] + (iy + 0.5) * g.pitch[1];
    const double inv_dt = 1.0 / f.dt;
    const double *qs = q + int64_t(iz) * f.n_ang * f.n_t;
    double acc = 0.0;
    for (int a = 0; a < f.n_ang; ++a) {
        const double t = -xc * sn[a] + yc * cs[a];
        const double s = (t - f.t0) * inv_dt - 0.5;
        const double fk = floor(s);
        const double w = s - fk;
        const double *row = qs + int64_t(a) * f.n_t;
        double q0 = 0.0, q1 = 0.0;
        if (fk >= 0.0 && fk < double(f.n_t)) q0 = row[int(fk)];
        if (fk >= -1.0 && fk < double(f.n_t - 1)) q1 = row[int(fk) + 1];
        acc += (1.0 - w) * q0 + w * q1;
    }
    x[int64_t(iz) * plane + v] = T(acc * (M_PI / f.n_ang));
}

// The same sum over 16 x 16 voxel tiles of kBpSlices slices.  Each angle's
// sine, cosine and window start are computed once per workgroup; then, chunk
// by chunk of angles, the workgroup stages in LDS the window of each slice's
// filtered row that the tile's lateral coordinates reach (zeros where the
// window runs past the row), so that the per-sample work has no bounds test
// and reads LDS only, and a thread's voxels at one (x, y) share the lateral
// coordinate, its bin and weight over the slices.  The next chunk's windows
// are loaded into registers while the current chunk is summed.  The lowest
// bin of angle a's window is one below floor(s) at the tile's lowest corner;
// its W bins cover the tile's whole lateral span (host bound) and the
// interpolation neighbour.  Same operations per voxel, same angle order and
// same zero rule as k_fbp_backproject.
// Grid: 8 * ceil(ngroups / 8) * tiles workgroups over ngroups = ceil(nz /
// kBpSlices) slice groups, placed on XCDs as there (group for slice).
// LDS: chunk * kBpSlices * W window bins, then n_ang sines, cosines and
// window starts; chunk * kBpSlices * W <= kBpPrefetch * kFbpWG.
constexpr int kBpTile = 16;
constexpr int kBpSlices = 4;
constexpr int kBpPrefetch = 16;           // window bins a thread holds for the next chunk
constexpr int kBpMaxWindow = 512;         // wider windows take k_fbp_backproject
constexpr int kBpAngleBytes = 2 * int(sizeof(double)) + int(sizeof(int));

template <typename T>
__global__ void __launch_bounds__(kFbpWG) k_fbp_backproject_tiled(const double *__restrict__ q, T *__restrict__ x,
                                                                  FbpDev f, GridDev g, int tiles_x, int tiles,
                                                                  int W, int chunk)
{
    extern __shared__ double lds[];
    const int span = kBpSlices * W;
    double *win = lds;                    // chunk * span bins
    double *cs = lds + int64_t(chunk) * span;
    double *sn = cs + f.n_ang;
    int *kb = reinterpret_cast<int *>(sn + f.n_ang);
    const int L = blockIdx.x;
    const int xcd = L % 8, j = L / 8;
    const int iz0 = kBpSlices * (xcd + 8 * (j / tiles));
    const int tile = j % tiles;
    if (iz0 >= g.n[2]) return;   // whole workgroup: no barrier below is skipped by part of it
    const int tx0 = (tile % tiles_x) * kBpTile, ty0 = (tile / tiles_x) * kBpTile;
    const int ux = tx0 + int(threadIdx.x) % kBpTile, uy = ty0 + int(threadIdx.x) / kBpTile;
    const bool mine = ux < g.n[0] && uy < g.n[1];
    // lanes past the grid's edge compute for the last voxel inside (never stored)
    const int ix = min(ux, g.n[0] - 1), iy = min(uy, g.n[1] - 1);
    const double xc = g.lo[0] + (ix + 0.5) * g.pitch[0];
    const double yc = g.lo[1] + (iy + 0.5) * g.pitch[1];
    // the tile's corner voxel centres bound every lane's lateral coordinate
    const double x0c = g.lo[0] + (tx0 + 0.5) * g.pitch[0];
    const double x1c = g.lo[0] + (min(tx0 + kBpTile, g.n[0]) - 0.5) * g.pitch[0];
    const double y0c = g.lo[1] + (ty0 + 0.5) * g.pitch[1];
    const double y1c = g.lo[1] + (min(ty0 + kBpTile, g.n[1]) - 0.5) * g.pitch[1];
    const double inv_dt = 1.0 / f.dt;
    for (int a = threadIdx.x; a < f.n_ang; a += blockDim.x) {
        double sa, ca;
        sincos(double(a) * f.dphi, &sa, &ca);
        sn[a] = sa;
        cs[a] = ca;
        const double t_lo = fmin(fmin(-x0c * sa + y0c * ca, -x1c * sa + y0c * ca),
                                 fmin(-x0c * sa + y1c * ca, -x1c * sa + y1c * ca));
        kb[a] = int(floor((t_lo - f.t0) * inv_dt - 0.5)) - 1;
    }
    __syncthreads();
    // the window bins of angles [a0, a0 + chunk) this thread stages: element e
    // = threadIdx.x + u * kFbpWG of the chunk's (angle, slice, bin) order
    double pre[kBpPrefetch];
    auto fetch = [&](int a0) {
        const int n = min(chunk, f.n_ang - a0) * span;
#pragma unroll
        for (int u = 0; u < kBpPrefetch; ++u) {
            const int e = int(threadIdx.x) + u * kFbpWG;
            double v = 0.0;
            if (e < n) {
                const int c = e / span;
                const int r = e - c * span;
                const int z = r / W;
                const int k = kb[a0 + c] + (r - z * W);
                // slices past the grid's end stage the last slice's rows (never stored)
                const int iz = min(iz0 + z, g.n[2] - 1);
                if (k >= 0 && k < f.n_t) v = q[(int64_t(iz) * f.n_ang + a0 + c) * f.n_t + k];
            }
            pre[u] = v;
        }
    };
    double acc[kBpSlices];
    for (int z = 0; z < kBpSlices; ++z) acc[z] = 0.0;
    fetch(0);
    for (int a0 = 0; a0 < f.n_ang; a0 += chunk) {
        const int na = min(chunk, f.n_ang - a0);
        __syncthreads();   // the previous chunk's windows are no longer read
#pragma unroll
        for (int u = 0; u < kBpPrefetch; ++u) {
            const int e = int(threadIdx.x) + u * kFbpWG;
            if (e < na * span) win[e] = pre[u];
        }
        __syncthreads();
        if (a0 + chunk < f.n_ang) fetch(a0 + chunk);
        for (int c = 0; c < na; ++c) {
            const int a = a0 + c;
            const double t = -xc * sn[a] + yc * cs[a];
            const double s = (t - f.t0) * inv_dt - 0.5;
            const double fk = floor(s);
            const double w = s - fk;
            // in [0, W - 2] by the window's construction; the clamp only keeps
            // the LDS reads inside the chunk
            const int i = min(max(int(fk) - kb[a], 0), W - 2);
            const double *row = win + c * span + i;
#pragma unroll
            for (int z = 0; z < kBpSlices; ++z) acc[z] += (1.0 - w) * row[z * W] + w * row[z * W + 1];
        }
    }
    if (!mine) return;
    const int64_t plane = int64_t(g.n[0]) * g.n[1];
    const int64_t v = int64_t(iy) * g.n[0] + ix;
#pragma unroll
    for (int z = 0; z < kBpSlices; ++z)
        if (iz0 + z < g.n[2]) x[int64_t(iz0 + z) * plane + v] = T(acc[z] * (M_PI / f.n_ang));
}

// Window width (bins) of a tile: its lateral span at any angle is at most
// (kBpTile - 1) (px + py) (|sin| <= 1, |cos| <= 1); the lowest bin sits one
// below the lowest corner's and the interpolation reads one past the
// highest, with a bin of margin for rounding.
// Geometries whose bin indices at the voxels could leave the int range (a
// far-off t0) take the untiled kernel too.
static int fbp_tile_window(const FbpDev &f, const GridDev &g)
{
    const double span = (kBpTile - 1) * (g.pitch[0] + g.pitch[1]) / f.dt;
    if (!(span < double(kBpMaxWindow))) return kBpMaxWindow + 1;
    const double r = std::hypot(std::max(std::fabs(g.lo[0]), std::fabs(g.hi[0])),
                                std::max(std::fabs(g.lo[1]), std::fabs(g.hi[1])));
    const double s_max = (r + std::fabs(f.t0)) / f.dt + 2.0;
    if (!(s_max < 1073741824.0)) return kBpMaxWindow + 1;
    return int(std::ceil(span)) + 5;
}

// Angles per chunk of the tiled kernel: the windows and every angle's sine,
// cosine and window start fit 32 KB of LDS (64 KB when the angles alone take
// more than 8 KB), and a thread holds at most kBpPrefetch of the next chunk's
// bins; 0 when not even one angle fits (k_fbp_backproject then).
static int fbp_tile_chunk(const FbpDev &f, int W)
{
    const int span_bytes = kBpSlices * W * int(sizeof(double));
    const int meta = f.n_ang * kBpAngleBytes;
    const int budget = meta <= 8192 ? 32768 : 65536;
    if (meta >= budget) return 0;
    return std::min({f.n_ang, (budget - meta) / span_bytes, kBpPrefetch * kFbpWG / (kBpSlices * W)});
}

static unsigned grid_stride_blocks(int64_t n)
{
    return unsigned(std::max<int64_t>(1, std::min<int64_t>(8192, (n + kFbpWG - 1) / kFbpWG)));
}

int launch_fbp_sinogram(const FbpDev &f, const ProtonsDev &p, int64_t n, const float *b, unsigned long long *sum,
                        unsigned *cnt, double *proj, int32_t *count, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nb = int64_t(f.nz) * f.n_ang * f.n_t;
    hipLaunchKernelGGL(k_fbp_clear, dim3(grid_stride_blocks(nb)), dim3(kFbpWG), 0, s, sum, cnt, nb);
    if (n > 0) {
        // privatised bins when one angle's (slice, lateral) bins fit the
        // workgroup's LDS on this device, else straight global atomics
        const size_t lds = size_t(f.nz) * f.n_t * sizeof(unsigned long long);
        int dev = 0, max_lds = 0;
        bool priv = hipGetDevice(&dev) == hipSuccess &&
                    hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
                    lds <= size_t(max_lds);
        if (priv && lds > 65536)
            priv = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fbp_bin_lds),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) == hipSuccess;
        (void)hipGetLastError();
        if (priv) {
            const int64_t chunk = std::min<int64_t>(kFbpMaxChunk, std::max<int64_t>(1024, (n + 1023) / 1024));
            hipLaunchKernelGGL(k_fbp_bin_lds, dim3(unsigned((n + chunk - 1) / chunk)), dim3(kFbpBinWG), lds, s, p, b, n,
                               chunk, f, sum, cnt);
        } else {
            hipLaunchKernelGGL(k_fbp_bin, dim3(grid_stride_blocks(n)), dim3(kFbpWG), 0, s, p, b, n, f, sum, cnt);
        }
    }
    hipLaunchKernelGGL(k_fbp_mean, dim3(grid_stride_blocks(nb)), dim3(kFbpWG), 0, s, sum, cnt, nb, proj, count);
    return hipGetLastError();
}

int launch_fbp_filter(const FbpDev &f, const double *proj, double *q, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t rows = int64_t(f.nz) * f.n_ang;
    // work items of a row: kFilterR-output groups of each parity; rows per
    // workgroup so that about kFbpWG items share it
    const int gpr = 2 * (((f.n_t + 1) / 2 + kFilterR - 1) / kFilterR);
    const int rpw = std::max(1, kFbpWG / gpr);
    const int ptaps = (f.n_t / 2 + kFilterR - 1) / kFilterR * kFilterR;
    const size_t lds = (size_t(ptaps) + size_t(rpw) * f.n_t) * sizeof(double);
    hipLaunchKernelGGL(k_fbp_filter, dim3(unsigned((rows + rpw - 1) / rpw)), dim3(kFbpWG), lds, s, proj, q, rows,
                       f.n_t, f.dt, rpw, gpr);
    return hipGetLastError();
}

int launch_fbp_backproject(const FbpDev &f, const GridDev &g, const double *q, void *x, int32_t dtype,
                           void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int W = fbp_tile_window(f, g);
    if (W <= kBpMaxWindow && fbp_tile_chunk(f, W) > 0) {
        const int tiles_x = (g.n[0] + kBpTile - 1) / kBpTile;
        const int tiles = tiles_x * ((g.n[1] + kBpTile - 1) / kBpTile);
        const int chunk = fbp_tile_chunk(f, W);
        const int groups = (g.n[2] + kBpSlices - 1) / kBpSlices;
        const unsigned grid = unsigned(8 * ((groups + 7) / 8) * int64_t(tiles));
        const size_t lds = size_t(chunk) * kBpSlices * W * sizeof(double) + size_t(f.n_ang) * kBpAngleBytes;
        if (dtype == PCT_F64)
            hipLaunchKernelGGL(k_fbp_backproject_tiled<double>, dim3(grid), dim3(kFbpWG), lds, s, q,
                               static_cast<double *>(x), f, g, tiles_x, tiles, W, chunk);
        else
            hipLaunchKernelGGL(k_fbp_backproject_tiled<float>, dim3(grid), dim3(kFbpWG), lds, s, q,
                               static_cast<float *>(x), f, g, tiles_x, tiles, W, chunk);
        return hipGetLastError();
    }
    const int64_t plane = int64_t(g.n[0]) * g.n[1];
    const int tiles = int((plane + kFbpWG - 1) / kFbpWG);
    const unsigned grid = unsigned(8 * ((g.n[2] + 7) / 8) * int64_t(tiles));
    const size_t lds = size_t(2) * f.n_ang * sizeof(double);
    if (dtype == PCT_F64)
        hipLaunchKernelGGL(k_fbp_backproject<double>, dim3(grid), dim3(kFbpWG), lds, s, q, static_cast<double *>(x),
                           f, g, tiles);
    else
        hipLaunchKernelGGL(k_fbp_backproject<float>, dim3(grid), dim3(kFbpWG), lds, s, q, static_cast<float *>(x), f,
                           g, tiles);
    return hipGetLastError();
}

}  // namespace pct
