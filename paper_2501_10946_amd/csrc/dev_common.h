// Device helpers shared by the kernels of librbsog.
#pragma once

#include <hip/hip_runtime.h>

#include "dev_math.h"
#include "launch.h"

namespace rbsog {

// Cell coordinate of a position: clamp(floor(x nc / L), 0, nc - 1); a NaN maps to 0.
__device__ inline int cell_coord(double x, double inv_cell, int nc)
{
    double f = floor(x * inv_cell);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)(nc - 1)) return nc - 1;
    return (int)f;
}

// Fixed-order sum over a 256-thread block; valid in thread 0.
__device__ inline double block_sum_256(double v, double *red)
{
    int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
#pragma unroll
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    return red[0];
}

}  // namespace rbsog
