// In-sample stream kernels for D = 1..4 (a translation unit of its own,
// so that the two halves compile in parallel).
#include "stream_dev.h"

namespace fjofc {

hipError_t launch_stream_lo(int D, int variant, int vec4, const InstDesc *insts,
                            const StreamItem *items, int nitems, int cur, bool stress,
                            bool acc, size_t lds, hipStream_t s) {
    switch (D) {
    case 1: return launch_stream_d<1>(variant, vec4, insts, items, nitems, cur, stress, acc, lds, s);
    case 2: return launch_stream_d<2>(variant, vec4, insts, items, nitems, cur, stress, acc, lds, s);
    case 3: return launch_stream_d<3>(variant, vec4, insts, items, nitems, cur, stress, acc, lds, s);
    case 4: return launch_stream_d<4>(variant, vec4, insts, items, nitems, cur, stress, acc, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fjofc
