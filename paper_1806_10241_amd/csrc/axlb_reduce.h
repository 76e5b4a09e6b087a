// Fixed-order FP64 block reduction shared by the reduction kernels.
// Internal to the HIP library.
#pragma once

#include <hip/hip_runtime.h>

namespace axlb {

constexpr int RED_THREADS = 256;

// Sums each of the K values over the workgroup (RED_THREADS threads): within
// each wavefront by shuffles, then the wavefront sums in order by thread 0,
// which holds the result.  The order never depends on scheduling, so the
// result is deterministic.  sh holds K * RED_THREADS / 64 doubles.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *sh) {
#pragma unroll
    for (int c = 0; c < K; ++c) {
        double x = v[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        v[c] = x;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < K; ++c) sh[c * (RED_THREADS / 64) + w] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int c = 0; c < K; ++c) {
            double s = 0.0;
            for (int k = 0; k < RED_THREADS / 64; ++k) s += sh[c * (RED_THREADS / 64) + k];
            v[c] = s;
        }
}

}  // namespace axlb
