// Internal declarations shared by the host entry points and the HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <vector>

#include "pct.h"

namespace pct {

// One table row per MLP vertex: c0t, c0th (mm), c2t, c2th (mm), u_k (mm), pad.
constexpr int kRowDoubles = 8;
constexpr int kMaxSegments = 1 << 16;
constexpr int kMaxUploads = 16;

// Geometry passed to kernels by value.
struct GridDev {
    int32_t n[3];
    double pitch[3];
    double inv_pitch[3];
    double inv_n[3];   // 1 / n and 1 / (nx ny): exact integer quotients by the extents
    double inv_nxy;
    double lo[3];  // origin
    double hi[3];  // origin + n*pitch
};

// How a proton's polyline is formed, passed to kernels by value.  Without a
// hull the vertices come from the shared coefficient table (K segments from
// tracker to tracker).  With a hull (the z-cylinder (x-hx)^2 + (y-hy)^2 <
// hr^2) each proton's most likely path runs between the points where its
// entry and exit tracks meet the hull, with its own coefficients, joined to
// the tracker planes by straight segments along the measured tracks.
struct PathSrc {
    const double *tab;  // (K+1) * kRowDoubles, shared table
    int K;              // tracker-to-tracker MLP segments
    int nvmax;          // most vertices a proton's polyline can have
    int hull;           // 0 or 1
    double hx, hy, hr;  // hull centre and radius (mm)
    double u_in, u_out, step;
    double poly[6], E0, X0;
    int log_term;
};

struct ProtonsDev {
    const float *t_in, *v_in, *th_in, *ph_in, *t_out, *v_out, *th_out, *ph_out, *gantry;
};

struct ProtonsBufDev {
    float *t_in, *v_in, *th_in, *ph_in, *t_out, *v_out, *th_out, *ph_out, *gantry;
};

// Workspace layout (byte offsets from the workspace base).
struct Layout {
    size_t hdr;      // status word and counters (256 B)
    size_t table;    // (K+1) * kRowDoubles doubles
    size_t acc;      // three block accumulators of (nvox + 4) 64-bit words
    size_t acc_stride;  // bytes between consecutive accumulators
    size_t cnt;      // nvox int32
    size_t x1;       // second copy of the iterate, nvox doubles
    size_t partial;  // kMaxPartials doubles
    size_t lo;       // compensation word of the FP32 iterate, nvox floats
    size_t total;    // end of the fixed part; the traced-ahead row slots and the bins follow

};
constexpr int kMaxPartials = 4096;
// One traced-ahead row record: 12 stash entries x 64 lanes of (voxel, chord),
// 64 lane counts and ||a_i||^2 (two slots of B records follow Layout::total).
constexpr size_t kSlotRecordBytes = size_t(12) * 64 * 8 + 64 * 4 + 8;
inline size_t slot_bytes(int64_t records) { return (size_t(records) * kSlotRecordBytes + 255) & ~size_t(255); }
// Slab bins of the binned schedule (after the two row slots): per slab of the
// block's dominant axis and row of the block, kBinCap entries (a packed
// 64-bit word each, the voxel index of entries 1.. in a second array) and, per
// block parity, the voxel index of entry 0 with the entry count in its top
// bits: 52 bytes per (slab, row); then the largest contribution of every row
// (one float per row).  Rows are rounded up to a multiple of 16;
// blocks of the binned schedule hold at most kBinMaxRows rows.
constexpr int kBinCap = 4;
constexpr int kBinMaxRows = 8192;
constexpr int kWinWords = 16384;  // LDS window of a slab commit: 128 KB of packed words
inline int64_t bin_rows(int64_t records) { return (records + 15) & ~int64_t(15); }
inline size_t bin_bytes(int64_t records, int nslab)
{
    const size_t nrow = size_t(nslab) * size_t(bin_rows(records));
    return (nrow * (kBinCap * 8 + (kBinCap - 1) * 4 + 2 * 4) + size_t(bin_rows(records)) * 4 + 255) & ~size_t(255);
}

// header words (int32 index): status word, then the [jmin, jmax] voxel range
// touched by a block, double-buffered by block parity (FP64 path), four
// rotating range slots of the fused FP32 path, the two overflow flags of the
// binned schedule (by block parity), and the block-boundary gate of
// cancellable calls: the host's cancel request, the gate word, the count of
// ended workgroups of the running commit launch and (int64) the block steps
// applied
enum : int {
    kHdrStatus = 0,
    kHdrRange0 = 2,
    kHdrRange1 = 4,
    kHdrSlots = 8,
    kHdrOvf = 16,
    kHdrCancel = 20,
    kHdrHalt = 21,
    kHdrGateCount = 22,
    kHdrDone = 24
};

Layout layout_for(int64_t nvox, int K, int dtype);

// FBP binning and back-projection geometry, passed to kernels by value.
struct FbpDev {
    int32_t n_ang, n_t, nz;
    double t0, dt, dphi;  // lateral bins [t0 + k dt, t0 + (k+1) dt); angle bin width 2 pi / n_ang
    double w;             // chord parameter of depth u = 0: -u_in / (u_out - u_in)
    double z0, pz;        // slice origin and thickness (mm)
};
constexpr double kFbpMaxWepl = 1048576.0;  // 2^20 mm: |b| at or beyond it is not a WEPL (dropped)
constexpr int kFbpMaxAngles = 4096;        // sines and cosines of every angle bin in LDS
constexpr int kFbpMaxLateral = 4096;       // a sinogram row and its filter taps in LDS

// FBP workspace layout (byte offsets): bin sums (int64 fixed point), bin
// counts (uint32), projections and filtered projections (double).
struct FbpLayout {
    size_t sum, cnt, proj, q, total;
};
FbpLayout fbp_layout(int64_t nbins);

}  // namespace pct

struct pct_plan {
    // serialises the host-side enqueue of DROP calls that share the plan (its
    // cached sweep graph, capture stream and profiling events)
    std::mutex mu;
    pct_grid grid;
    pct_mlp mlp;
    int K;
    int64_t nvox;
    std::vector<double> table;  // (K+1) * kRowDoubles
    void *uploaded[pct::kMaxUploads];
    int n_uploaded;
    // profiling events (hipEvent_t), pairs per sampled launch and kernel kind
    std::vector<void *> prof_events[2];
    int prof_used[2];
    // instantiated graph of one DROP sweep (hipGraphExec_t) and its launch key
    void *graph_exec;
    std::vector<uint64_t> graph_key;
    void *capture_stream;  // private hipStream_t used only to record the graph
    void *cancel_stream;   // private hipStream_t that writes cancel requests
    int hull;              // 1: per-proton MLP between the hull entry and exit points
    double hull_c[2], hull_r;
};

namespace pct {

// Launchers implemented in the HIP translation unit.  They assume validated
// arguments and return a hipError_t value.
PathSrc path_src(const pct_plan &pl, const void *table_dev);
int path_vertices_max(const pct_plan &pl);
int launch_trace(const pct_plan &pl, const ProtonsDev &p, int64_t first, int64_t count, int32_t max_nnz,
                 int32_t *vox, double *chord, int32_t *nnz, void *ws, void *stream);
int launch_forward(const pct_plan &pl, const ProtonsDev &p, int64_t n, const void *x, int dtype, void *y,
                   void *nrm2, void *ws, void *stream);
int launch_backproject(const pct_plan &pl, const ProtonsDev &p, int64_t n, const void *r, int dtype, void *g,
                       void *ws, void *stream);
int launch_drop(pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, void *x,
                const pct_drop_opts &o, void *ws, size_t ws_bytes, void *stream);
int launch_rows_count(const pct_plan &pl, const ProtonsDev &p, int64_t n, int64_t *offsets, void *ws, void *stream);
int launch_rows_build(const pct_plan &pl, const ProtonsDev &p, int64_t n, int chord_type, const int64_t *offsets,
                      int32_t *vox, void *chord, double *n2, void *ws, void *stream);
int launch_drop_rows(pct_plan &pl, const pct_rows &rows, const float *b, float *x, const pct_drop_opts &o, void *ws,
                     void *stream);
int launch_span_histogram(const pct_plan &pl, const ProtonsDev &p, int64_t n, int64_t *hist, void *stream);
int launch_order_blocks(const pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, int64_t block,
                        const ProtonsBufDev &out, float *b_out, void *stream);
int copy_device(void *dst, const void *src, size_t bytes, void *stream);
int launch_region_select(const pct_plan &pl, const ProtonsDev &p, int64_t n, const float *b, int z_lo, int z_hi,
                         const ProtonsBufDev &out, int64_t capacity, float *b_out, int64_t *count, void *ws,
                         void *stream);
int launch_tv(const pct_plan &pl, const void *x, int dtype, double eps, double *value_dev, void *grad, void *ws,
              void *stream);
int launch_tv_static(const pct_plan &pl, const void *x, int dtype, double eps, double *value_dev, void *grad,
                     void *stream);
int upload_table(const pct_plan &pl, void *ws, void *stream);
int launch_fbp_sinogram(const FbpDev &f, const ProtonsDev &p, int64_t n, const float *b, unsigned long long *sum,
                        unsigned *cnt, double *proj, int32_t *count, void *stream);
int launch_fbp_filter(const FbpDev &f, const double *proj, double *q, void *stream);
int launch_fbp_backproject(const FbpDev &f, const GridDev &g, const double *q, void *x, int32_t dtype,
                           void *stream);
int profile_read(pct_plan &pl, double ms[2], int64_t launches[2]);
void profile_release(pct_plan &pl);
void graph_release(pct_plan &pl);
int read_status(const pct_plan &pl, void *ws, int reset, uint32_t *bits, void *stream);
int write_cancel(pct_plan &pl, void *ws, int32_t request);
int read_progress(const pct_plan &pl, void *ws, int64_t *done, int *halted, void *stream);
int launch_gate_reset(const pct_plan &pl, void *ws, void *stream);

GridDev grid_dev(const pct_grid &g);

}  // namespace pct
