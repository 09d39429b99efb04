// Wavefront-level helpers shared by the out-of-sample and cMDS kernels
// (gfx950: 64-lane wavefronts, DPP row operations, permlane swaps).
#pragma once
#include <hip/hip_runtime.h>

namespace fjofc {
namespace wave {

constexpr int DPP_QP_XOR1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QP_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_ROR8 = 0x128;

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Lanes 0-31 return a summed over both 32-lane halves, lanes 32-63 return b.
__device__ __forceinline__ float swap32_add(float a, float b) {
    auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
// Even 16-lane rows return a summed over the row pair, odd rows return b.
__device__ __forceinline__ float swap16_add(float a, float b) {
    auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

// Reduce V values (V % 8 == 0) over the 64 lanes.  Afterwards c[r] in every
// lane of an aligned group of 8 lanes holds the wave total of value
//   r + bit3 V/8 + bit4 V/4 + bit5 V/2     (bits of the lane index).
template <int V>
__device__ __forceinline__ void reduce_scatter8(float (&p)[V], float (&c)[V / 8], int lane) {
    static_assert(V % 8 == 0, "V is a multiple of 8");
    float a[V / 2];
#pragma unroll
    for (int r = 0; r < V / 2; ++r) a[r] = swap32_add(p[r], p[r + V / 2]);
    float b[V / 4];
#pragma unroll
    for (int r = 0; r < V / 4; ++r) b[r] = swap16_add(a[r], a[r + V / 4]);
    const bool b3 = lane & 8;
#pragma unroll
    for (int r = 0; r < V / 8; ++r) {
        const float send = b3 ? b[r] : b[r + V / 8];
        const float keep = b3 ? b[r + V / 8] : b[r];
        c[r] = keep + dpp<DPP_ROW_ROR8>(send);
    }
#pragma unroll
    for (int r = 0; r < V / 8; ++r) {
        c[r] += dpp<DPP_QP_XOR1>(c[r]);
        c[r] += dpp<DPP_QP_XOR2>(c[r]);
        c[r] += dpp<DPP_ROW_HALF_MIRROR>(c[r]);
    }
}

// Index of the value a lane holds in c[r] after reduce_scatter8<V>.
__device__ __forceinline__ int scatter8_base(int lane, int V) {
    return ((lane >> 3) & 1) * (V / 8) + ((lane >> 4) & 1) * (V / 4) + ((lane >> 5) & 1) * (V / 2);
}

}  // namespace wave
}  // namespace fjofc
