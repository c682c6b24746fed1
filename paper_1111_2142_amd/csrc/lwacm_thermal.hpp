// lwacm_thermal.hpp -- arguments and launch of the temperature-lattice step
// (thermal LW-ACM, Eq. ACM2.0t with the even part of Eq. feqe).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lwacm {

constexpr int kMaxThermalWallIds = 16;

struct ThermalArgs {
    int Q, nx, ny, nz;
    int QT;               // temperature lattice: Q, or 5 (D2Q5) / 7 (D3Q7), the rest
                          // and axis links of the flow's lattice
    float kap;            // 2 - 2/omega_t: weight of the even-part difference
    float h;              // 1 - kap = 2/omega_t - 1
    const void *state;    // flow state at the step's time (storage format: D + 1 values per node)
    int st_half;          // state in FP16 deviations (lwacm storage LWACM_FP16_DEV)
    float ld_scale[2];    // storage -> value factors of (rho - 1, u); 1 for FP32
    const float *T_in;    // T at the step's time
    float *T_out;         // T one step later
    const uint8_t *mask;  // 0 fluid, m >= 1 solid with wall id m; null: no walls
    float wall_T[kMaxThermalWallIds];  // temperature of wall id m; NaN: adiabatic
};

hipError_t launch_thermal_step(const ThermalArgs &t, hipStream_t stream);

// For the temperature step fused into the D3Q19 flow kernel with walls: per
// node, the links i whose upstream node x - v_i is a wall held at a fixed
// temperature (bit i, the flow kernels' link order) and the FP32 bits of the
// sum of 36 w_i T_w over them; zero for solid nodes and away from such walls.
hipError_t launch_thermal_wall_table(const ThermalArgs &t, uint2 *out, hipStream_t stream);

// Reverse mode of one temperature step (lwacm_adjoint_thermal_step).
struct ThermalAdjArgs {
    ThermalArgs t;         // the step's arguments; t.state and t.T_in are its inputs
    const float *lam_in;   // dL/dT(t + 1)
    float *lam_out;        // dL/dT(t) through this step
    float *mu;             // the flow cotangent dL/du(t) is added to (see the header)
    int final_t0;          // mu field-major (the gradient of the initial state)
};

hipError_t launch_thermal_adjoint(const ThermalAdjArgs &a, hipStream_t stream);

}  // namespace lwacm
