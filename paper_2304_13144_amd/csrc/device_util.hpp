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

// Partial sums of eq. 1 over chunks of SUM_CHUNK consecutive atoms:
// part[chunk][0] = sum V_i, part[chunk][1 + k] = sum W_i,k (virial component
// k), zero where the input is NULL.  Called by a whole block of 256 threads
// for one chunk: wavefront w takes atoms 8 w .. 8 w + 7 of the chunk, lane l
// atom l / 8 and the values l % 8 and 8 + l % 8; shuffles add the eight
// atoms of a wavefront, then the four wavefronts are added in order.
constexpr int SUM_CHUNK = 32;
__device__ inline void chunk_partials(int64_t chunk, int64_t n, const double *site_e, const double *vir,
                                      double *part) {
    __shared__ double sp[4][10];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, s = lane & 7;
    const int64_t i = chunk * SUM_CHUNK + 8 * w + (lane >> 3);
    double v0 = 0.0, v1 = 0.0;   // value s and value 8 + s (0: V_i, 1 + k: W_i,k)
    if (i < n) {
        if (s == 0) v0 = site_e ? site_e[i] : 0.0;
        else v0 = vir ? vir[9 * i + s - 1] : 0.0;
        if (s < 2) v1 = vir ? vir[9 * i + 7 + s] : 0.0;
    }
#pragma unroll
    for (int o = 8; o < 64; o <<= 1) {
        v0 += __shfl_xor(v0, o, 64);
        v1 += __shfl_xor(v1, o, 64);
    }
    if (lane < 8) sp[w][lane] = v0;
    if (lane < 2) sp[w][8 + lane] = v1;
    __syncthreads();
    if (threadIdx.x < 10) {
        const int t = threadIdx.x;
        part[chunk * 10 + t] = ((sp[0][t] + sp[1][t]) + sp[2][t]) + sp[3][t];
    }
}

}  // namespace mtp
