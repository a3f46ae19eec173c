// Mode algebra of the gradient workload: the initial velocity
//   u0 = u_base + sum_m a_m B_m
// (velocity modes added to the Taylor-Green velocity) and the projection of
// an adjoint velocity field on the mode fields, dL/da_m = <B_m, dL/du0>.
// The projection is deterministic: fixed-order block sums, then one block
// adds the block partials in block order.
#include <hip/hip_runtime.h>

#include "sllbm_internal.h"

namespace sllbm {

namespace {

constexpr int PCHUNK = 8;   // modes per projection pass

__global__ void __launch_bounds__(256) k_superpose(int64_t n, int m, ModeAmplitudes am,
                                                   const double *__restrict__ base,
                                                   const double *__restrict__ basis, double *__restrict__ out)
{
    for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s = fma(am.a[j], basis[j * n + k], s);
        out[k] = base[k] + s;
    }
}

__device__ __forceinline__ void block_tree(double (&v)[PCHUNK], double *red)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < PCHUNK; ++j) red[j * 256 + tid] = v[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int j = 0; j < PCHUNK; ++j) red[j * 256 + tid] += red[j * 256 + tid + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < PCHUNK; ++j) v[j] = red[j * 256];
}

// partials[block][j] = sum over the block's components of B_{m0+j} v (j < mc)
__global__ void __launch_bounds__(256) k_project_partial(int64_t n, int m0, int mc, const double *__restrict__ basis,
                                                         const double *__restrict__ v, double *__restrict__ partials)
{
    __shared__ double red[PCHUNK * 256];
    double acc[PCHUNK];
#pragma unroll
    for (int j = 0; j < PCHUNK; ++j) acc[j] = 0.0;
    for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double vk = v[k];
#pragma unroll
        for (int j = 0; j < PCHUNK; ++j)
            if (j < mc) acc[j] = fma(basis[(m0 + j) * n + k], vk, acc[j]);
    }
    block_tree(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < PCHUNK; ++j) partials[blockIdx.x * PCHUNK + j] = acc[j];
    }
}

// out[j] = sum of partials[b][j] over the blocks: thread t adds blocks t,
// t + 256, ... in order, then a fixed tree
__global__ void __launch_bounds__(256) k_project_final(const double *__restrict__ partials, int nblocks,
                                                       double *__restrict__ out)
{
    __shared__ double red[PCHUNK * 256];
    double acc[PCHUNK];
#pragma unroll
    for (int j = 0; j < PCHUNK; ++j) acc[j] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
        for (int j = 0; j < PCHUNK; ++j) acc[j] += partials[b * PCHUNK + j];
    block_tree(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < PCHUNK; ++j) out[j] = acc[j];
    }
}

int grid_of(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return static_cast<int>(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace

hipError_t launch_superpose(int64_t n, int m, const ModeAmplitudes &am, const double *base, const double *basis,
                            double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_superpose, dim3(grid_of(n)), dim3(256), 0, st, n, m, am, base, basis, out);
    return hipGetLastError();
}

hipError_t launch_project_chunk(int64_t n, int m0, int mc, const double *basis, const double *v, double *partials,
                                int nblocks, double *out8, hipStream_t st)
{
    hipLaunchKernelGGL(k_project_partial, dim3(nblocks), dim3(256), 0, st, n, m0, mc, basis, v, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_project_final, dim3(1), dim3(256), 0, st, partials, nblocks, out8);
    return hipGetLastError();
}

}  // namespace sllbm
