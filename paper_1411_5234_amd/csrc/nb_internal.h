// Internal declarations shared by the HIP translation units of libnbody.so:
// what the kernels are compiled against.  The host-side context is in ctx.h.
//
// Every kernel of the block-step path works from a table of Items: one Item per
// system taking part in the launch, plus an array `starts` of n_items + 1
// workgroup offsets (item k owns workgroups [starts[k], starts[k+1])).  A
// single-system call is a table of one item, so the arithmetic a system sees
// does not depend on what else is in the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nbody.h"

// Bits of a status word latched by kernels.
enum : int {
    NBK_ERANGE = 1,   // a new step fell below dt_min
    NBK_ENAN = 2,     // non-finite acceleration, jerk or step
    NBK_EINDEX = 4,   // active index out of range
};

// Small fixed-size device area of a context.
struct nb_small {
    int status;          // the context's status word
    int pad;
    double energy[2];
};

namespace nbk {

#ifndef NBK_TILE
#define NBK_TILE 512
#endif
#ifndef NBK_UNROLL
#define NBK_UNROLL 2
#endif
#ifndef NBK_FOLD
#define NBK_FOLD 32
#endif

constexpr int WG = 256;          // threads per workgroup (4 waves of 64)
constexpr int TILE = NBK_TILE;   // j-bodies per LDS tile

// One system's part of a launch.  Plain data, uploaded to the device.
struct Item {
    nb_system s;                 // the system's arrays
    const int32_t *i_idx;        // active list, or null for i = k
    double *acc, *jerk;          // force outputs / corrector inputs, rows c*m + k
    double *snap;                // 6th order: third output / input, else null
    nb_hermite6 h6;              // 6th order: snap, crackle, predicted acceleration
    double *part;                // force partials of this item (j_chunks > 1)
    int *status;                 // error word
    double eps2;                 // softening squared
    double t_next;               // block time
    int64_t j0, j1;              // force j-range
    int64_t chunk;               // j per chunk (a multiple of the kernel's work granule)
    int32_t m;                   // active block size
    int32_t b;                   // j-chunks (Bfactor)
    int64_t sel_slice;           // selection: bodies per workgroup
    int64_t sel_off;             // selection: first slot of this item's temporaries
    int32_t sel_blocks;          // selection: workgroups
    int32_t red_lanes;           // partial reduction: lanes per output value
    double *tensor;              // tidal tensor output, rows (3a+b)*nrows + row
    double *t_out;               // tidal: time of each listed body (or null)
    int64_t row0;                // tidal: output row = i - row0 (bodies below skipped), or k if < 0
    int64_t nrows;               // tidal: row stride of the output
    const double *pts;           // tidal at points: 3 * nrows coordinates (x, then y, then z), or null
    const int32_t *excl;         // tidal at points: 2 * nrows rows left out (-1: none), or null
    int32_t *nn;                 // nearest: neighbour of each listed body (-1: not searched)
    double *r2;                  // nearest: its squared distance
    int64_t row_end;             // nearest: listed bodies at or above this row are not searched
    double dt_cap;               // nearest: listed bodies with a larger step are not searched
};

// Per-item selection results written by the selection kernels.
struct SelResult {
    double t_next;
    int32_t m;
    int32_t status;
};

struct Table {
    const Item *items;           // device
    const int64_t *starts;       // device, n + 1 entries
    int n;
    int64_t blocks;              // starts[n]
};

// Item owning workgroup `blk`: the largest k with starts[k] <= blk.
__device__ __forceinline__ int find_item(const int64_t *starts, int n, int64_t blk)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Outputs per active body: 6 (acc, jerk) or 9 (acc, jerk, snap).
__host__ __device__ inline int force_outputs(const Item &it) { return it.snap ? 9 : 6; }

}  // namespace nbk
