// The plain fused over-relaxation substep (arXiv:1211.0780, Eq. (2)) for
// gfx950: the instantiations of the kernel template in xy_or2_kernel.h that
// do not measure.  A translation unit of its own because it is compiled with
// the max-ILP instruction scheduler (the build script's per-source flags),
// which takes the substep from 0.2202-0.2206 to 0.2167-0.2172 ms at
// L = 160 x 32 replicas.
#include <hip/hip_runtime.h>

#include "xy_kernels.h"
#include "xy_or2_kernel.h"

namespace xy {

hipError_t launch_or2_plain(bool lead, int spt, int grid, size_t lds, const SweepArgs &a, hipStream_t s,
                            int *per_cu)
{
    return launch_or2_lead<kOr2Plain>(lead, spt, grid, lds, a, s, per_cu);
}

}  // namespace xy
