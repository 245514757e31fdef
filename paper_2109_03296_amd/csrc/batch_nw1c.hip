// Batched persistent search kernel, 1 wavefront per workgroup, waves take contiguous shares of an item's velocities.
#include "batch_kernels.h"

namespace kbm {
namespace batch {

hipError_t launch_batch_nw1c(const BatchLaunch &l, unsigned grid, hipStream_t stream) {
    hipLaunchKernelGGL((batch_kernel<1, true>), dim3(grid), dim3(WAVE * 1), 0, stream,
                       l.descs, l.info, l.pre, l.seg, l.ctrl, l.prog, l.nseg, l.vbs, l.st_x,
                       l.st_y);
    return hipGetLastError();
}

hipError_t occupancy_nw1c(int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, reinterpret_cast<const void *>(&batch_kernel<1, true>), WAVE * 1, 0);
}

}  // namespace batch
}  // namespace kbm
