// Kernels of the inverse-problem layer: the BiLaplacian prior's elliptic
// operator (paper Sec. 2) and the vector updates and float64 dot products of
// the Newton-CG iteration (Sec. 4).
//
// Prior operator, cell-centred on the solver's grid:
//   (A u)_i = alpha (u_i - sum over the faces of cell i of theta_a (u_nb - u_i) / dx^2),
// faces on the domain boundary carry no flux (zero normal flux of Theta grad u).
// All of these kernels stream their vectors once; they are HBM-bound and cost
// microseconds beside the solves of a gradient or a Hessian-vector product.

#include "wv_internal.h"

namespace wv {

namespace {

constexpr int DB = 256;  // dot-product block size

int grid_for(long long n, int bs)
{
    long long g = (n + bs - 1) / bs;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

// out = scale A (u - u0) (+ out when accumulate); u0 may be null (taken as 0).
// One thread per cell, x fastest so every access of a wavefront is coalesced;
// the z and y neighbours are the planes just read by the neighbouring work-groups
// and come from L2.
__global__ void prior_kernel(const float* __restrict__ u, const float* __restrict__ u0, float* __restrict__ out,
                             int nz, int ny, int nx, float alpha, float cz, float cy, float cx, float scale,
                             int accumulate)
{
    const long long plane = (long long)ny * nx;
    const long long N = plane * nz;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < N;
         q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % nx);
        const long long t = q / nx;
        const int j = (int)(t % ny);
        const int k = (int)(t / ny);
        auto val = [&](long long r) { return u0 ? u[r] - u0[r] : u[r]; };
        const float w = val(q);
        float flux = 0.f;
        if (k > 0) flux += cz * (val(q - plane) - w);
        if (k < nz - 1) flux += cz * (val(q + plane) - w);
        if (j > 0) flux += cy * (val(q - nx) - w);
        if (j < ny - 1) flux += cy * (val(q + nx) - w);
        if (i > 0) flux += cx * (val(q - 1) - w);
        if (i < nx - 1) flux += cx * (val(q + 1) - w);
        const float a = scale * (alpha * (w - flux));
        out[q] = accumulate ? out[q] + a : a;
    }
}

// y = a x + b y
__global__ void axpby_kernel(float* __restrict__ y, const float* __restrict__ x, float a, float b, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        y[q] = a * x[q] + b * y[q];
}

// out = x + a y
__global__ void lincomb_kernel(float* __restrict__ out, const float* __restrict__ x, float a,
                               const float* __restrict__ y, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        out[q] = x[q] + a * y[q];
}

__device__ inline double dblock_sum(double v)
{
    __shared__ double sh[DB / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < DB / 64; ++q) r += sh[q];
    __syncthreads();
    return r;
}

// fixed-order two-stage float64 dot product (bitwise reproducible)
__global__ void dot_kernel(const float* __restrict__ a, const float* __restrict__ b, long long n,
                           double* __restrict__ partial)
{
    double acc = 0.0;
    for (long long q = blockIdx.x * (long long)DB + threadIdx.x; q < n; q += (long long)gridDim.x * DB)
        acc += (double)a[q] * (double)b[q];
    const double t = dblock_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void dot_finalize(const double* __restrict__ partial, int n, double* __restrict__ out)
{
    double acc = 0.0;
    for (int q = threadIdx.x; q < n; q += DB) acc += partial[q];
    const double t = dblock_sum(acc);
    if (threadIdx.x == 0) out[0] = t;
}

}  // namespace

void launch_prior(const float* u, const float* u0, float* out, int nz, int ny, int nx, double alpha, double cz,
                  double cy, double cx, double scale, bool accumulate, hipStream_t st)
{
    const long long N = (long long)nz * ny * nx;
    hipLaunchKernelGGL(prior_kernel, dim3(grid_for(N, 256)), dim3(256), 0, st, u, u0, out, nz, ny, nx, (float)alpha,
                       (float)cz, (float)cy, (float)cx, (float)scale, accumulate ? 1 : 0);
    WV_HIP(hipGetLastError());
}

void launch_axpby(float* y, const float* x, double a, double b, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, y, x, (float)a, (float)b, n);
    WV_HIP(hipGetLastError());
}

void launch_lincomb(float* out, const float* x, double a, const float* y, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, out, x, (float)a, y, n);
    WV_HIP(hipGetLastError());
}

void launch_dot(const float* a, const float* b, long long n, double* partial, int nblocks, double* d_out,
                hipStream_t st)
{
    hipLaunchKernelGGL(dot_kernel, dim3(nblocks), dim3(DB), 0, st, a, b, n, partial);
    hipLaunchKernelGGL(dot_finalize, dim3(1), dim3(DB), 0, st, partial, nblocks, d_out);
    WV_HIP(hipGetLastError());
}

}  // namespace wv
