// lwacm_force.hpp -- force and torque on a wall by momentum exchange.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lwacm {

constexpr unsigned kForceBlock = 256;
constexpr unsigned kForceMaxBlocks = 4096;

struct ForceArgs {
    int Q, nx, ny, nz;
    float A;               // 3 (2/omega - 1)
    const float *state;    // FP32 state, D + 1 floats per node
    const uint8_t *mask;   // 0 fluid, m >= 1 solid with wall id m
    const float *qd;       // link-wall distances (Q fields) or null: halfway walls
    int wall_id;
    double xc[3];          // torque centre (node coordinates)
    double *partials;      // [6 * nblocks]
    double *out;           // [6]: F, T
    const unsigned *list;  // fluid nodes next to a wall (node order), or null: scan every node
    unsigned nlist;
};

// Launches the pass over the listed nodes (or over every node when list is
// null) on nblocks blocks and the fixed-order sum.
hipError_t launch_wall_force(const ForceArgs &f, unsigned nblocks, hipStream_t stream);

}  // namespace lwacm
