// lwacm_walls.hpp -- the list of fluid nodes next to a wall and the per-step
// wall correction of the D3Q19 tile kernel (host-side declarations).
#pragma once

#include <hip/hip_runtime.h>

#include "lwacm_internal.hpp"

namespace lwacm {

// Blocks (and counts) of the list build for n nodes.
size_t wall_list_count_blocks(long long n);
// Counts per block of 256 nodes, scanned in place into offsets; the total
// goes to *d_total (device).  Then the scatter writes the node indices in
// node order into list (total entries).
hipError_t launch_wall_list_count(const ProblemArgs &p, unsigned *counts,
                                  unsigned long long *d_total, hipStream_t s);
hipError_t launch_wall_list_scatter(const ProblemArgs &p, const unsigned *offsets,
                                    unsigned *list, hipStream_t s);
// The wall links of the listed nodes, as the correction kernel reads them.
struct WallLinks {
    const unsigned *list;    // listed nodes (node order)
    unsigned nlist;
    const unsigned *bits;    // per entry: bit i set when x - v_i is solid
    const float *qc;         // 18 * nlist: q of incoming link i of entry k at (i - 1) * nlist + k
    const unsigned *second;  // per entry: bit i when the q < 1/2 rule takes x + v_i
    int table_moving;        // the per-id table has a moving wall
};
// Packs qc, second and the entries' link sets from d_q and the mask (once per context: the walls,
// like the mask, are fixed for its life).  D3Q19 only.
hipError_t launch_wall_pack(const ProblemArgs &p, const unsigned *list, unsigned nlist, float *qc,
                            unsigned *second, unsigned *wbits, hipStream_t s);
// corr[x] for every listed node: the interpolated bounce-back minus the
// halfway term plus the whole moving-wall term, summed with 36 w_i into
// (1, v_i), from the state src (storage format).  D3Q19 only.
hipError_t launch_wall_correction(const ProblemArgs &p, int storage, const void *src,
                                  const WallLinks &w, float4 *corr, hipStream_t s);

}  // namespace lwacm
