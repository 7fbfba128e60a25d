// Sum of a matrix and its transpose: y = x + x^T, float64 (arXiv 2101.08878,
// Section V-B, "Sum of cuPy Array and its Transpose": the benchmark adds a
// chunked cuPy array to its transpose).
//
// HBM-bound: every element of x is read once and every element of y written
// once.  The matrix is cut into 32 x 32 tiles; a workgroup takes one tile
// pair (I, J) with I <= J, stages tiles x[I, J] and x[J, I] in LDS (rows
// padded by one element, so that reading a column touches consecutive
// banks), then writes y[I, J] = x[I, J] + x[J, I]^T and y[J, I] = x[J, I] +
// x[I, J]^T.  Both tiles are read before either is written, so y may be x.
// Each element is one IEEE-754 addition, the same on any device.
#include "mdx.h"
#include "mdx_internal.hpp"

namespace mdx {
namespace {

// 32 x 32 tiles, 256 threads: 17 KB of LDS per workgroup, so many
// workgroups share a CU and keep loads in flight (4.9 TB/s at 16K x 16K,
// against 2.6 TB/s for 64 x 64 tiles at two workgroups per CU).
constexpr int kTT = 32;                    // tile edge
constexpr int kTThreads = 256;
constexpr int kTRows = kTThreads / kTT;    // rows a workgroup moves per step
static_assert(kTT % kTRows == 0, "tile rows split evenly over the steps");

// Tile pair of workgroup p: pairs are numbered row by row over I <= J, so
// row I starts at I T - I (I - 1) / 2.
__device__ __forceinline__ void pair_of(int64_t p, int64_t T, int64_t &I, int64_t &J)
{
    const double b = 2.0 * (double)T + 1.0;
    int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)p)) * 0.5);
    i = i < 0 ? 0 : (i >= T ? T - 1 : i);
    auto start = [T](int64_t r) { return r * T - r * (r - 1) / 2; };
    while (i > 0 && start(i) > p)
        --i;
    while (i + 1 < T && start(i + 1) <= p)
        ++i;
    I = i;
    J = i + (p - start(i));
}

__global__ __launch_bounds__(kTThreads) void transpose_sum_tiles(const double *x, double *y, int64_t n,
                                                             int64_t T)
{
    __shared__ double a[kTT][kTT + 1], b[kTT][kTT + 1];
    int64_t I, J;
    pair_of(blockIdx.x, T, I, J);
    const int c = threadIdx.x % kTT, r0 = threadIdx.x / kTT;
    const int64_t i0 = I * kTT, j0 = J * kTT;
    const bool diag = I == J;
#pragma unroll
    for (int k = 0; k < kTT / kTRows; ++k) {
        const int r = r0 + k * kTRows;
        const int64_t ra = i0 + r, ca = j0 + c;  // x[I, J]
        if (ra < n && ca < n)
            a[r][c] = x[ra * n + ca];
        const int64_t rb = j0 + r, cb = i0 + c;  // x[J, I]
        if (!diag && rb < n && cb < n)
            b[r][c] = x[rb * n + cb];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTT / kTRows; ++k) {
        const int r = r0 + k * kTRows;
        const int64_t ra = i0 + r, ca = j0 + c;
        if (ra < n && ca < n)
            y[ra * n + ca] = a[r][c] + (diag ? a[c][r] : b[c][r]);
        const int64_t rb = j0 + r, cb = i0 + c;
        if (!diag && rb < n && cb < n)
            y[rb * n + cb] = b[r][c] + a[c][r];
    }
}

}  // namespace

hipError_t launch_transpose_sum(const double *x, double *y, int64_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const int64_t T = (n + kTT - 1) / kTT;
    const int64_t pairs = T * (T + 1) / 2;
    trace_begin("transpose_sum", s);
    hipLaunchKernelGGL(transpose_sum_tiles, dim3((unsigned)pairs), dim3(kTThreads), 0, s, x, y, n, T);
    trace_end("transpose_sum", s);
    return hipGetLastError();
}

}  // namespace mdx
