// Device sort of an acquisition-order scan into angle bins.  Section IV-A of
// the paper reconstructs a scan taken with continuous gantry rotation; its
// records arrive in acquisition order and are grouped by angle bin, then by a
// slab of the entry height v_in, then by the lateral entry t_in, so that a
// block of consecutive records covers neighbouring paths.
//
// Each record gets a 64-bit key  a << (32 + bits_s) | s << 32 | ord(t_in)
// (ord: the FP32 bit pattern mapped so that unsigned order is numeric order,
// with -0 taken as +0; a non-finite record gets a = n_angles and sorts last),
// and the (key, position) pairs go through a least-significant-digit radix
// sort with 8-bit digits, one pass per digit the key uses:
//
//   k_sort_keys         one thread per record: the key, the position, and a
//                       packed 40-byte copy of the record (9 fields and b)
//   k_sort_hist         one workgroup per tile of 2048 pairs: digit counts in
//                       LDS, written digit-major (count of digit d in tile g at
//                       d * n_tiles + g), so that one exclusive scan of the
//                       counts gives every (digit, tile) its output offset
//   k_sort_count_*      that scan: partial sums of 4096 counts, a one-workgroup
//                       scan of the partials, then the scan of each segment
//   k_sort_scatter      one workgroup per tile, 8 rounds of 256 pairs in input
//                       order: a lane's rank among the lanes of its wave with
//                       the same digit comes from 8 ballots (one per digit
//                       bit), the counts of earlier waves and rounds from LDS;
//                       equal digits keep their input order (stable).  The
//                       tile's pairs are staged in LDS in digit order and
//                       written out as one run per digit
//   k_sort_gather       one thread per output record: copy the record from its
//                       input position, read from the packed copy (the angles
//                       of a continuous scan are uniform in acquisition order,
//                       so sources are random: one or two cache lines per
//                       record instead of one per field)
//
// The sort is integer work: the output is unique and bit-exact whatever the
// launch shape.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <utility>

#include "pct_sort.h"

namespace pct {

namespace {

constexpr int kSortWG = 256;
constexpr int kSortWaves = kSortWG / 64;
constexpr int kSortRounds = 8;
constexpr int64_t kSortTile = int64_t(kSortWG) * kSortRounds;   // records per tile
constexpr int kScanPer = 16;
constexpr int64_t kScanSeg = int64_t(kSortWG) * kScanPer;       // counts per scan workgroup

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__device__ inline unsigned long long sort_key(const SortDev &s, float phi32, float v32, float t32)
{
    if (!isfinite(phi32) || !isfinite(v32) || !isfinite(t32))
        return static_cast<unsigned long long>(s.n_angles) << (32 + s.bits_s);
    // angle bin: nearest bin centre a * dphi, taken modulo the turn (fa is an
    // integer, so the remainder is exact)
    const double fa = floor(double(phi32) / s.dphi + 0.5);
    double r = fmod(fa, double(s.n_angles));
    if (r < 0.0) r += double(s.n_angles);
    const unsigned a = unsigned(r);
    const double fs = floor((double(v32) - s.z0) / s.slab);
    const unsigned sl = fs <= 0.0 ? 0u : (fs >= double(s.n_slabs - 1) ? unsigned(s.n_slabs - 1) : unsigned(fs));
    unsigned u = __float_as_uint(t32 == 0.0f ? 0.0f : t32);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return (static_cast<unsigned long long>(a) << (32 + s.bits_s)) | (static_cast<unsigned long long>(sl) << 32) |
           static_cast<unsigned long long>(u);
}

__global__ void __launch_bounds__(kSortWG) k_sort_keys(ProtonsDev p, const float *b, int64_t n, SortDev s,
                                                       unsigned long long *key, uint32_t *idx, float *rec)
{
    // the workgroup's packed records are staged in LDS and written out as
    // 16-byte stores over its contiguous 10 * 256 floats
    __shared__ float4 stage[kSortWG * 10 / 4];
    float *st = reinterpret_cast<float *>(stage);
    const int64_t i0 = int64_t(blockIdx.x) * kSortWG;
    const int64_t i = i0 + threadIdx.x;
    if (i < n) {
        const float t = p.t_in[i], v = p.v_in[i], phi = p.gantry[i];
        key[i] = sort_key(s, phi, v, t);
        idx[i] = uint32_t(i);
        float *r = st + 10 * threadIdx.x;
        r[0] = t;
        r[1] = v;
        r[2] = p.th_in[i];
        r[3] = p.ph_in[i];
        r[4] = p.t_out[i];
        r[5] = p.v_out[i];
        r[6] = p.th_out[i];
        r[7] = p.ph_out[i];
        r[8] = phi;
        r[9] = b ? b[i] : 0.0f;
    }
    __syncthreads();
    const int count = int(min<int64_t>(kSortWG, n - i0));     // records of this workgroup
    const int nf = 10 * count;                                  // floats to write
    float *out = rec + 10 * i0;                                 // 16-byte aligned: 10 * 256 floats per workgroup
    for (int q = threadIdx.x; q < nf / 4; q += kSortWG) reinterpret_cast<float4 *>(out)[q] = stage[q];
    for (int q = (nf / 4) * 4 + threadIdx.x; q < nf; q += kSortWG) out[q] = st[q];
}

__global__ void __launch_bounds__(kSortWG) k_sort_hist(const unsigned long long *key, int64_t n, int shift,
                                                       int64_t n_tiles, uint32_t *hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t tile0 = int64_t(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = tile0 + int64_t(r) * kSortWG + threadIdx.x;
        if (i < n) atomicAdd(&h[unsigned(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[int64_t(threadIdx.x) * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive prefix sum of v over the workgroup in thread order; total gets
// the sum.  lds: kSortWG words.
__device__ inline uint32_t wg_exclusive_scan(uint32_t v, uint32_t *lds, uint32_t &total)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kSortWG; off <<= 1) {
        const uint32_t a = t >= off ? lds[t - off] : 0u;
        __syncthreads();
        lds[t] += a;
        __syncthreads();
    }
    const uint32_t incl = lds[t];
    total = lds[kSortWG - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kSortWG) k_sort_count_reduce(const uint32_t *hist, int64_t nh, uint32_t *part)
{
    __shared__ uint32_t lds[kSortWG];
    const int64_t seg = int64_t(blockIdx.x) * kScanSeg;
    uint32_t sum = 0;
    for (int j = 0; j < kScanPer; ++j) {
        const int64_t e = seg + int64_t(j) * kSortWG + threadIdx.x;
        if (e < nh) sum += hist[e];
    }
    uint32_t total;
    wg_exclusive_scan(sum, lds, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kSortWG) k_sort_count_top(uint32_t *part, int64_t np)
{
    __shared__ uint32_t lds[kSortWG];
    const int64_t per = (np + kSortWG - 1) / kSortWG;
    const int64_t lo = min(np, int64_t(threadIdx.x) * per);
    const int64_t hi = min(np, lo + per);
    uint32_t sum = 0;
    for (int64_t e = lo; e < hi; ++e) sum += part[e];
    uint32_t total;
    uint32_t run = wg_exclusive_scan(sum, lds, total);
    for (int64_t e = lo; e < hi; ++e) {
        const uint32_t v = part[e];
        part[e] = run;
        run += v;
    }
}

__global__ void __launch_bounds__(kSortWG) k_sort_count_down(uint32_t *hist, int64_t nh, const uint32_t *part)
{
    __shared__ uint32_t lds[kSortWG];
    const int64_t first = int64_t(blockIdx.x) * kScanSeg + int64_t(threadIdx.x) * kScanPer;
    uint32_t v[kScanPer];
    uint32_t sum = 0;
    for (int j = 0; j < kScanPer; ++j) {
        const int64_t e = first + j;
        v[j] = e < nh ? hist[e] : 0u;
        sum += v[j];
    }
    uint32_t total;
    uint32_t run = part[blockIdx.x] + wg_exclusive_scan(sum, lds, total);
    for (int j = 0; j < kScanPer; ++j) {
        const int64_t e = first + j;
        if (e < nh) hist[e] = run;
        run += v[j];
    }
}

__global__ void __launch_bounds__(kSortWG) k_sort_scatter(const unsigned long long *key_in, const uint32_t *idx_in,
                                                          int64_t n, int shift, int64_t n_tiles, const uint32_t *off,
                                                          unsigned long long *key_out, uint32_t *idx_out)
{
    __shared__ uint32_t base[256];                  // next output slot of each digit
    __shared__ uint32_t first[256];                 // output slot of the tile's first pair of each digit
    __shared__ uint32_t local[256];                 // tile-local start of each digit (pairs in digit order)
    __shared__ uint32_t cnt[kSortWaves][256];       // this round's count per wave and digit
    __shared__ unsigned long long skey[kSortTile];  // the tile's pairs, staged in digit order
    __shared__ uint32_t sidx[kSortTile];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    // pairs of digit t in this tile: the next offset of the scanned counts
    // (digit-major) minus this one; the last entry ends at n
    const int64_t e = int64_t(t) * n_tiles + blockIdx.x;
    const uint32_t o0 = off[e];
    const uint32_t o1 = e + 1 < 256 * n_tiles ? off[e + 1] : uint32_t(n);
    base[t] = o0;
    first[t] = o0;
    for (int w = 0; w < kSortWaves; ++w) cnt[w][t] = 0;
    uint32_t tile_total;
    local[t] = wg_exclusive_scan(o1 - o0, cnt[0], tile_total);   // cnt[0] is scratch here, cleared below
    cnt[0][t] = 0;
    __syncthreads();
    const int64_t tile0 = int64_t(blockIdx.x) * kSortTile;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = tile0 + int64_t(r) * kSortWG + t;
        const bool valid = i < n;
        unsigned long long k = 0;
        uint32_t ix = 0;
        if (valid) {
            k = key_in[i];
            ix = idx_in[i];
        }
        const unsigned d = unsigned(k >> shift) & 255u;
        unsigned long long same = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const unsigned long long m = __ballot((d >> bit) & 1u);
            same &= ((d >> bit) & 1u) ? m : ~m;
        }
        const uint32_t rank = uint32_t(__popcll(same & below));
        if (valid && rank == 0) cnt[wave][d] = uint32_t(__popcll(same));
        __syncthreads();
        if (valid) {
            uint32_t dst = base[d] + rank;
            for (int w = 0; w < wave; ++w) dst += cnt[w][d];
            const uint32_t lp = local[d] + (dst - first[d]);
            if (lp < uint32_t(kSortTile)) {
                skey[lp] = k;
                sidx[lp] = ix;
            }
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kSortWaves; ++w) {
            add += cnt[w][t];
            cnt[w][t] = 0;
        }
        base[t] += add;
        __syncthreads();
    }
    // write the staged pairs out in digit order: consecutive threads write
    // consecutive slots of each digit's run
    for (uint32_t q = uint32_t(t); q < tile_total && q < uint32_t(kSortTile); q += kSortWG) {
        const unsigned long long k = skey[q];
        const unsigned d = unsigned(k >> shift) & 255u;
        const uint32_t dst = first[d] + (q - local[d]);
        if (int64_t(dst) < n) {
            key_out[dst] = k;
            idx_out[dst] = sidx[q];
        }
    }
}

__global__ void __launch_bounds__(kSortWG) k_sort_gather(const float *rec, int64_t n, const uint32_t *idx,
                                                         ProtonsBufDev o, float *b_out, int64_t *perm)
{
    const int64_t j = int64_t(blockIdx.x) * kSortWG + threadIdx.x;
    if (j >= n) return;
    const int64_t i = idx[j];
    if (i >= n) return;                 // idx is a permutation of 0 .. n-1
    const float2 *r = reinterpret_cast<const float2 *>(rec + 10 * i);
    const float2 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4];
    o.t_in[j] = r0.x;
    o.v_in[j] = r0.y;
    o.th_in[j] = r1.x;
    o.ph_in[j] = r1.y;
    o.t_out[j] = r2.x;
    o.v_out[j] = r2.y;
    o.th_out[j] = r3.x;
    o.ph_out[j] = r3.y;
    o.gantry[j] = r4.x;
    if (b_out) b_out[j] = r4.y;
    if (perm) perm[j] = i;
}

}  // namespace

SortLayout sort_layout(int64_t n)
{
    SortLayout L{};
    L.n_tiles = (n + kSortTile - 1) / kSortTile;
    L.n_hist = 256 * L.n_tiles;
    L.n_parts = (L.n_hist + kScanSeg - 1) / kScanSeg;
    size_t o = 0;
    L.keys0 = o;
    o += align256(size_t(n) * 8);
    L.keys1 = o;
    o += align256(size_t(n) * 8);
    L.idx0 = o;
    o += align256(size_t(n) * 4);
    L.idx1 = o;
    o += align256(size_t(n) * 4);
    L.hist = o;
    o += align256(size_t(L.n_hist) * 4);
    L.part = o;
    o += align256(size_t(L.n_parts) * 4);
    L.rec = o;
    o += align256(size_t(n) * 40);
    L.total = o;
    return L;
}

int launch_sort_scan(const SortDev &s, const ProtonsDev &p, int64_t n, const float *b, const ProtonsBufDev &o,
                     float *b_out, int64_t *perm, void *ws, void *stream)
{
    if (n <= 0) return hipSuccess;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const SortLayout L = sort_layout(n);
    char *w = static_cast<char *>(ws);
    auto *k0 = reinterpret_cast<unsigned long long *>(w + L.keys0);
    auto *k1 = reinterpret_cast<unsigned long long *>(w + L.keys1);
    auto *i0 = reinterpret_cast<uint32_t *>(w + L.idx0);
    auto *i1 = reinterpret_cast<uint32_t *>(w + L.idx1);
    auto *hist = reinterpret_cast<uint32_t *>(w + L.hist);
    auto *part = reinterpret_cast<uint32_t *>(w + L.part);
    auto *rec = reinterpret_cast<float *>(w + L.rec);
    const unsigned blocks = unsigned((n + kSortWG - 1) / kSortWG);
    hipLaunchKernelGGL(k_sort_keys, dim3(blocks), dim3(kSortWG), 0, st, p, b, n, s, k0, i0, rec);
    for (int pass = 0; pass < s.passes; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_hist, dim3(unsigned(L.n_tiles)), dim3(kSortWG), 0, st, k0, n, shift, L.n_tiles,
                           hist);
        hipLaunchKernelGGL(k_sort_count_reduce, dim3(unsigned(L.n_parts)), dim3(kSortWG), 0, st, hist, L.n_hist,
                           part);
        hipLaunchKernelGGL(k_sort_count_top, dim3(1), dim3(kSortWG), 0, st, part, L.n_parts);
        hipLaunchKernelGGL(k_sort_count_down, dim3(unsigned(L.n_parts)), dim3(kSortWG), 0, st, hist, L.n_hist, part);
        hipLaunchKernelGGL(k_sort_scatter, dim3(unsigned(L.n_tiles)), dim3(kSortWG), 0, st, k0, i0, n, shift,
                           L.n_tiles, hist, k1, i1);
        std::swap(k0, k1);
        std::swap(i0, i1);
    }
    hipLaunchKernelGGL(k_sort_gather, dim3(blocks), dim3(kSortWG), 0, st, rec, n, i0, o, b_out, perm);
    return hipGetLastError();
}

}  // namespace pct
