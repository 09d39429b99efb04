// The persistent batched kernel for batches whose largest D is at most
// 8 (its own translation unit, so that the two tiers compile in parallel).
#include "batch_dev.h"

namespace fjofc {

hipError_t launch_batch_kernel8(const BatchArgs &a, int grid, size_t lds, hipStream_t s) {
    batch_kernel<8><<<dim3((unsigned)grid), dim3(BATCH_BLOCK), lds, s>>>(a);
    return hipGetLastError();
}

const void *batch_kernel8_address() {
    return reinterpret_cast<const void *>(&batch_kernel<8>);
}

}  // namespace fjofc
