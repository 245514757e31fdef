// Batched persistent search kernel, 4 wavefronts per workgroup, waves take contiguous shares of an item's velocities.
#include "batch_kernels.h"

namespace kbm {
namespace batch {

hipError_t launch_batch_nw4c(const BatchLaunch &l, unsigned grid, hipStream_t stream) {
    hipLaunchKernelGGL((batch_kernel<4, true>), dim3(grid), dim3(WAVE * 4), 0, stream,
                       l.descs, l.info, l.pre, l.seg, l.ctrl, l.prog, l.nseg, l.vbs, l.st_x,
                       l.st_y);
    return hipGetLastError();
}

hipError_t occupancy_nw4c(int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, reinterpret_cast<const void *>(&batch_kernel<4, true>), WAVE * 4, 0);
}

}  // namespace batch
}  // namespace kbm
