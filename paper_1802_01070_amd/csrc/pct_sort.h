// Device sort of an acquisition-order scan into angle bins (continuous gantry
// rotation, Section IV-A): internal interface between the C-ABI and the HIP
// kernels of pct_sort.hip.
#pragma once

#include <cstddef>
#include <cstdint>

#include "pct_internal.h"

namespace pct {

struct SortDev {
    int32_t n_angles;   // angle bins; n_angles itself marks a non-finite record
    int32_t n_slabs;    // slabs of the entry height v_in
    int32_t bits_s;     // key bits of the slab field
    int32_t passes;     // 8-bit digit passes over the key
    double dphi;        // 2 pi / n_angles
    double z0;          // lower z edge of the grid
    double slab;        // slab thickness (mm)
};

// Workspace layout (byte offsets, each 256-byte aligned)
struct SortLayout {
    size_t keys0, keys1, idx0, idx1, hist, part;
    size_t rec;         // n packed records of 10 floats (9 fields, then b)
    size_t total;
    int64_t n_tiles;    // tiles of kSortTile records
    int64_t n_hist;     // 256 * n_tiles digit counts
    int64_t n_parts;    // partial sums of the count scan
};

constexpr int32_t kSortMaxAngles = 4096;
constexpr int32_t kSortMaxSlabs = 4096;
constexpr int64_t kSortMaxRecords = (int64_t(1) << 31) - 1;

SortLayout sort_layout(int64_t n);
int launch_sort_scan(const SortDev &s, const ProtonsDev &p, int64_t n, const float *b, const ProtonsBufDev &o,
                     float *b_out, int64_t *perm, void *ws, void *stream);

}  // namespace pct
