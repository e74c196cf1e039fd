// Small device-side helpers shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mtp {

// Inclusive scan over a block of NT threads (s: NT ints of LDS); the last
// element, s[NT - 1], is the block total on return.
template <int NT> __device__ inline int32_t block_scan(int32_t v, int32_t *s) {
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < NT; d <<= 1) {
        const int32_t t = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    return s[threadIdx.x];
}

}  // namespace mtp
