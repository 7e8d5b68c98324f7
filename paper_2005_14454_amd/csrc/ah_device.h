// Device-side helpers shared by the HIP translation units of libah.
#pragma once

#include "ah_internal.h"

namespace ah {

// Fold nblocks diagnostics records (kMeasStride doubles each) into
// out[0 .. M_COUNT) with 256 threads in a fixed order: thread t sums records
// t, t+256, ... in turn, then a fixed pairwise tree.  Sums except M_GMAX,
// which is max-reduced.  `red` is 256 doubles of LDS.  Call with 256 threads.
__device__ inline void fold_records(const double* __restrict__ partials, int nblocks, double* __restrict__ out,
                                    double* red)
{
    for (int k = 0; k < M_COUNT; ++k) {
        double r = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += 256) {
            const double v = partials[(int64_t)b * kMeasStride + k];
            r = (k == M_GMAX) ? fmax(r, v) : r + v;
        }
        red[threadIdx.x] = r;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                red[threadIdx.x] = (k == M_GMAX) ? fmax(red[threadIdx.x], red[threadIdx.x + w])
                                                 : red[threadIdx.x] + red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

}  // namespace ah
