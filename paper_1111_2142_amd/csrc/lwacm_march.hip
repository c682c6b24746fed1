// lwacm_march.hip -- D3Q19 z-marching tile kernel (placeholder: the generic
// kernel serves every problem until this kernel lands).
#include "lwacm_internal.hpp"

namespace lwacm {

bool march_supported(const ProblemArgs &) { return false; }

unsigned march_num_blocks(const ProblemArgs &) { return 0; }

hipError_t launch_fwd_march(const ProblemArgs &, int, bool, const void *, void *,
                            const ReduceArgs &, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace lwacm
