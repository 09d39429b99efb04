// In-sample stream kernels for D = 5..8 (a translation unit of its own,
// so that the two halves compile in parallel).
#include "stream_dev.h"

namespace fjofc {

hipError_t launch_stream_hi(int D, int variant, int vec4, const InstDesc *insts,
                            const StreamItem *items, int nitems, int cur, bool stress,
                            bool acc, size_t lds, hipStream_t s) {
    switch (D) {
    case 5: return launch_stream_d<5>(variant, vec4, insts, items, nitems, cur, stress, acc, lds, s);
    case 6: return launch_stream_d<6>(variant, vec4, insts, items, nitems, cur, stress, acc, lds, s);
    case 7: return launch_stream_d<7>(variant, vec4, insts, items, nitems, cur, stress, acc, lds, s);
    case 8: return launch_stream_d<8>(variant, vec4, insts, items, nitems, cur, stress, acc, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fjofc
