// Volume transpose for the forward sweeps: the tiles that sweep x planes
// stage their boxes from a copy of the volume with x and y swapped, so that
// a box row (fixed z, in-plane index y) is contiguous in memory.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

namespace cbct {
namespace {

// out[s][x][y] = in[s][y][x] for the n_slices (channel x z) slices of a
// volume: 32 x 32 tiles through LDS, both sides' accesses along rows.
template <class T>
__global__ void __launch_bounds__(256)
transpose_xy(const T *__restrict__ in, T *__restrict__ out, int nx, int ny, int n_slices)
{
    __shared__ T tile[32][33];
    const int tx = (nx + 31) >> 5;
    const int x0 = (blockIdx.x % tx) * 32, y0 = (blockIdx.x / tx) * 32;
    const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;   // 32 x 8
    const size_t plane = (size_t)nx * ny;
    for (int sl = blockIdx.y; sl < n_slices; sl += gridDim.y) {
        const T *src = in + sl * plane;
        T *dst = out + sl * plane;
        __syncthreads();   // the previous slice's readers of the tile are done
#pragma unroll
        for (int j = ly; j < 32; j += 8) {
            const int x = x0 + lx, y = y0 + j;
            if (x < nx && y < ny)
                tile[j][lx] = src[(size_t)y * nx + x];
        }
        __syncthreads();
#pragma unroll
        for (int j = ly; j < 32; j += 8) {
            const int y = y0 + lx, x = x0 + j;
            if (x < nx && y < ny)
                dst[(size_t)x * ny + y] = tile[lx][j];
        }
    }
}

// Launch transpose_xy over n_slices slices of nx x ny elements.
template <class T>
inline void launch_transpose_xy(const T *in, T *out, int nx, int ny, int n_slices, hipStream_t s)
{
    const dim3 grid(((nx + 31) / 32) * ((ny + 31) / 32), std::min(n_slices, 65535));
    hipLaunchKernelGGL((transpose_xy<T>), grid, dim3(256), 0, s, in, out, nx, ny, n_slices);
}

}  // namespace
}  // namespace cbct
