// The persistent batched kernel for batches whose largest D is at most
// 5 (its own translation unit, so that the two tiers compile in parallel).
#include "batch_dev.h"

namespace fjofc {

hipError_t launch_batch_kernel5(const BatchArgs &a, int grid, size_t lds, hipStream_t s) {
    batch_kernel<5><<<dim3((unsigned)grid), dim3(BATCH_BLOCK), lds, s>>>(a);
    return hipGetLastError();
}

const void *batch_kernel5_address() {
    return reinterpret_cast<const void *>(&batch_kernel<5>);
}

}  // namespace fjofc
