// Small device-side helpers shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mtp {

// "Last block" completion: every block calls this after writing its partial
// results; it returns true in exactly one block, the last to arrive, which
// then sees every other block's writes.  The ticket must be zero before the
// launch; the last block resets it (reset_ticket), so back-to-back launches
// and graph replays need no memset.
__device__ inline bool last_block(unsigned *ticket) {
    __shared__ bool is_last;
    __threadfence();   // publish this block's writes before taking a ticket
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = atomicAdd(ticket, 1u);
        is_last = t == gridDim.x * gridDim.y * gridDim.z - 1;
    }
    __syncthreads();
    if (is_last) __threadfence();   // order the reads of the other blocks' writes after the ticket
    return is_last;
}

__device__ inline void reset_ticket(unsigned *ticket) {
    if (threadIdx.x == 0) atomicExch(ticket, 0u);
}

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
