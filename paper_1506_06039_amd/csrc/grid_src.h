// The searched grid's values read from where they live: an FP64 grid, or a
// frame's pixels with the grid value formed as it is read.  Device code only
// (included by the HIP sources).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace moco {

// SRC: 0 FP64 grid [mg][ng]; 1 uint16 pixels [m][n], 2x2 box mean; 2 uint16
// pixels as they are; 3 float pixels, 2x2 box mean; 4 float pixels as they are.
// The box means are the grid kernels' values: for uint16 a quarter of the
// integer sum (exact), for float ((x00 + x01) + x10) + x11 in FP64, over 4.
template <int SRC>
__device__ __forceinline__ const void *grid_frame(const void *src, size_t f, int m, int n,
                                                  int mg, int ng)
{
    if (SRC == 0) return (const double *)src + f * mg * ng;
    if (SRC <= 2) return (const uint16_t *)src + f * m * n;
    return (const float *)src + f * m * n;
}

template <int SRC>
__device__ __forceinline__ double grid_at(const void *a, int n, int ng, int i, int j)
{
    if (SRC == 0) return ((const double *)a)[(size_t)i * ng + j];
    if (SRC == 1) {
        const uint16_t *p = (const uint16_t *)a + (size_t)(2 * i) * n + 2 * j;
        return 0.25 * (double)((int)p[0] + (int)p[1] + (int)p[n] + (int)p[n + 1]);
    }
    if (SRC == 2) return (double)((const uint16_t *)a)[(size_t)i * n + j];
    if (SRC == 3) {
        const float *p = (const float *)a + (size_t)(2 * i) * n + 2 * j;
        const double x00 = (double)p[0], x01 = (double)p[1];
        const double x10 = (double)p[n], x11 = (double)p[n + 1];
        return (((x00 + x01) + x10) + x11) / 4.0;
    }
    return (double)((const float *)a)[(size_t)i * n + j];
}

}  // namespace moco
