// Element-wise and reduction kernels: c^2, misfit with float64 accumulation,
// gradient assembly from the Kahan accumulators, comparisons and norms.
// Reductions are two-stage (fixed-order block partials, then one block) so
// results are bitwise reproducible.

#include "wv_internal.h"

namespace wv {

namespace {

constexpr int RB = 256;  // reduction block size

__device__ inline double block_sum(double v)
{
    __shared__ double sh[RB / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < RB / 64; ++q) r += sh[q];
    __syncthreads();
    return r;
}

__global__ void square_kernel(const float* __restrict__ c, float* __restrict__ m, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const float v = c[q];
        m[q] = v * v;
    }
}

__global__ void misfit_kernel(const float* __restrict__ p, const float* __restrict__ d,
                              float* __restrict__ resid, long long n, double wres,
                              double* __restrict__ partial)
{
    double acc = 0.0;
    for (long long q = blockIdx.x * (long long)RB + threadIdx.x; q < n; q += (long long)gridDim.x * RB) {
        const double diff = (double)p[q] - (double)d[q];
        acc += diff * diff;
        resid[q] = (float)(wres * diff);
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void finalize_kernel(const double* __restrict__ partial, int n, double scale,
                                double* __restrict__ out)
{
    double acc = 0.0;
    for (int q = threadIdx.x; q < n; q += RB) acc += partial[q];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) out[0] = scale * t;
}

__global__ void scale_kernel(const float* __restrict__ p, float* __restrict__ out, long long n, double w)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        out[q] = (float)(w * (double)p[q]);
}

// g = scale * c * sum_s (acc_s - cmp_s)
__global__ void grad_finish_kernel(const float* __restrict__ c, const float* __restrict__ acc,
                                   long long N, int nsrc, double scale, float* __restrict__ g)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < N;
         q += (long long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nsrc; ++k) {
            const float* a = acc + (long long)k * 2 * N;
            s += (double)a[q] - (double)a[N + q];
        }
        g[q] = (float)(scale * (double)c[q] * s);
    }
}

// -2 dt (dc * sum_s acc_s + c * sum_s dacc_s), each sum as (sum - compensation) in float64
__global__ void newton_finish_kernel(const float* __restrict__ c, const float* __restrict__ dc,
                                     const float* __restrict__ acc, const float* __restrict__ dacc, long long N,
                                     int nsrc, double scale, float* __restrict__ h)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < N;
         q += (long long)gridDim.x * blockDim.x) {
        double s = 0.0, ds = 0.0;
        for (int k = 0; k < nsrc; ++k) {
            s += (double)acc[(long long)k * 2 * N + q] - (double)acc[(long long)k * 2 * N + N + q];
            ds += (double)dacc[(long long)k * 2 * N + q] - (double)dacc[(long long)k * 2 * N + N + q];
        }
        h[q] = (float)(scale * ((double)dc[q] * s + (double)c[q] * ds));
    }
}

__global__ void fill_kernel(float* __restrict__ p, long long n, float v)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        p[q] = v;
}

__global__ void copy_kernel(float* __restrict__ dst, const float* __restrict__ src, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        dst[q] = src[q];
}

__global__ void compare_kernel(const float* __restrict__ a, const float* __restrict__ b, long long n,
                               int* __restrict__ flag)
{
    int bad = 0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        bad |= (__float_as_uint(a[q]) != __float_as_uint(b[q]));
    if (bad) atomicOr(flag, 1);
}

// partial sums of (a-b)^2 and b^2 for a relative L2 error
__global__ void rel_err_kernel(const float* __restrict__ a, const float* __restrict__ b, long long n,
                               double* __restrict__ partial)
{
    double e = 0.0, r = 0.0;
    for (long long q = blockIdx.x * (long long)RB + threadIdx.x; q < n; q += (long long)gridDim.x * RB) {
        const double d = (double)a[q] - (double)b[q];
        e += d * d;
        r += (double)b[q] * (double)b[q];
    }
    const double te = block_sum(e);
    const double tr = block_sum(r);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = te;
        partial[2 * blockIdx.x + 1] = tr;
    }
}

__global__ void rel_err_finalize(const double* __restrict__ partial, int n, double* __restrict__ out)
{
    double e = 0.0, r = 0.0;
    for (int q = threadIdx.x; q < n; q += RB) {
        e += partial[2 * q];
        r += partial[2 * q + 1];
    }
    const double te = block_sum(e);
    const double tr = block_sum(r);
    if (threadIdx.x == 0) out[0] = tr > 0.0 ? sqrt(te / tr) : sqrt(te);
}

// both sums of rel_err_kernel's partials: out[0] = sum (a - b)^2, out[1] = sum b^2
__global__ void err_norms_finalize(const double* __restrict__ partial, int n, double* __restrict__ out)
{
    double e = 0.0, r = 0.0;
    for (int q = threadIdx.x; q < n; q += RB) {
        e += partial[2 * q];
        r += partial[2 * q + 1];
    }
    const double te = block_sum(e);
    const double tr = block_sum(r);
    if (threadIdx.x == 0) {
        out[0] = te;
        out[1] = tr;
    }
}

// per-field max |x| over a stack of states [nstates][4][N]; one block row per field
__global__ void absmax_kernel(const float* __restrict__ st, long long nstates, long long N,
                              double* __restrict__ partial)
{
    const int f = blockIdx.y;
    float mx = 0.f;
    const long long total = nstates * N;
    for (long long q = blockIdx.x * (long long)RB + threadIdx.x; q < total; q += (long long)gridDim.x * RB) {
        const long long sidx = q / N, c = q - sidx * N;
        mx = fmaxf(mx, fabsf(st[(sidx * 4 + f) * N + c]));
    }
    __shared__ float sh[RB];
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int o = RB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[f * gridDim.x + blockIdx.x] = sh[0];
}

__global__ void absmax_finalize(const double* __restrict__ partial, int nb, double* __restrict__ out)
{
    const int f = threadIdx.x;
    if (f < 4) {
        double m = 0.0;
        for (int q = 0; q < nb; ++q) m = fmax(m, partial[f * nb + q]);
        out[f] = m;
    }
}

__global__ void range_kernel(const float* __restrict__ x, long long n, double* __restrict__ partial)
{
    float lo = INFINITY, hi = -INFINITY;
    unsigned nan = 0;
    for (long long q = blockIdx.x * (long long)RB + threadIdx.x; q < n; q += (long long)gridDim.x * RB) {
        const float v = x[q];
        if (v != v) ++nan;
        else { lo = fminf(lo, v); hi = fmaxf(hi, v); }
    }
    __shared__ float slo[RB], shi[RB];
    __shared__ unsigned snan[RB];
    slo[threadIdx.x] = lo; shi[threadIdx.x] = hi; snan[threadIdx.x] = nan;
    __syncthreads();
    for (int o = RB / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            slo[threadIdx.x] = fminf(slo[threadIdx.x], slo[threadIdx.x + o]);
            shi[threadIdx.x] = fmaxf(shi[threadIdx.x], shi[threadIdx.x + o]);
            snan[threadIdx.x] += snan[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x] = slo[0];
        partial[3 * blockIdx.x + 1] = shi[0];
        partial[3 * blockIdx.x + 2] = snan[0];
    }
}

__global__ void range_finalize(const double* __restrict__ partial, int nb, double* __restrict__ out)
{
    if (threadIdx.x == 0) {
        double lo = INFINITY, hi = -INFINITY, nan = 0.0;
        for (int q = 0; q < nb; ++q) {
            lo = fmin(lo, partial[3 * q]);
            hi = fmax(hi, partial[3 * q + 1]);
            nan += partial[3 * q + 2];
        }
        out[0] = lo; out[1] = hi; out[2] = nan;
    }
}

__global__ void dm_kernel(const float* __restrict__ c, const float* __restrict__ dc, float* __restrict__ dm,
                          long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        dm[q] = 2.0f * c[q] * dc[q];
}

int grid_for(long long n, int bs)
{
    long long g = (n + bs - 1) / bs;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

void launch_square(const float* c, float* m, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(square_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, c, m, n);
    WV_HIP(hipGetLastError());
}

void launch_misfit(const float* p, const float* d, float* resid, long long n, double wres, double wJ,
                   double* partial, int nblocks, double* d_out, hipStream_t st)
{
    hipLaunchKernelGGL(misfit_kernel, dim3(nblocks), dim3(RB), 0, st, p, d, resid, n, wres, partial);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(RB), 0, st, partial, nblocks, wJ, d_out);
    WV_HIP(hipGetLastError());
}

void launch_scale_weights(const float* p, float* resid, long long n, double w, hipStream_t st)
{
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, resid, n, w);
    WV_HIP(hipGetLastError());
}

void launch_newton_finish(const float* c, const float* dc, const float* acc, const float* dacc, long long N,
                          int nsrc, double scale, float* h, hipStream_t st)
{
    hipLaunchKernelGGL(newton_finish_kernel, dim3(grid_for(N, 256)), dim3(256), 0, st, c, dc, acc, dacc, N, nsrc,
                       scale, h);
    WV_HIP(hipGetLastError());
}

void launch_grad_finish(const float* c, const float* acc, long long N, int nsrc, double scale, float* g,
                        hipStream_t st)
{
    hipLaunchKernelGGL(grad_finish_kernel, dim3(grid_for(N, 256)), dim3(256), 0, st, c, acc, N, nsrc,
                       scale, g);
    WV_HIP(hipGetLastError());
}

void launch_fill(float* p, long long n, float v, hipStream_t st)
{
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
    WV_HIP(hipGetLastError());
}

void launch_copy(float* dst, const float* src, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, dst, src, n);
    WV_HIP(hipGetLastError());
}

void launch_compare(const float* a, const float* b, long long n, int* flag, hipStream_t st)
{
    hipLaunchKernelGGL(compare_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, a, b, n, flag);
    WV_HIP(hipGetLastError());
}

void launch_rel_err(const float* a, const float* b, long long n, double* partial, int nblocks,
                    double* d_out, hipStream_t st)
{
    hipLaunchKernelGGL(rel_err_kernel, dim3(nblocks), dim3(RB), 0, st, a, b, n, partial);
    hipLaunchKernelGGL(rel_err_finalize, dim3(1), dim3(RB), 0, st, partial, nblocks, d_out);
    WV_HIP(hipGetLastError());
}

void launch_err_norms(const float* a, const float* b, long long n, double* partial, int nblocks, double* d_out2,
                      hipStream_t st)
{
    hipLaunchKernelGGL(rel_err_kernel, dim3(nblocks), dim3(RB), 0, st, a, b, n, partial);
    hipLaunchKernelGGL(err_norms_finalize, dim3(1), dim3(RB), 0, st, partial, nblocks, d_out2);
    WV_HIP(hipGetLastError());
}

void launch_range(const float* x, long long n, double* partial, int nblocks, double* d_out3,
                  hipStream_t st)
{
    hipLaunchKernelGGL(range_kernel, dim3(nblocks), dim3(RB), 0, st, x, n, partial);
    hipLaunchKernelGGL(range_finalize, dim3(1), dim3(64), 0, st, partial, nblocks, d_out3);
    WV_HIP(hipGetLastError());
}

void launch_dm(const float* c, const float* dc, float* dm, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(dm_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, c, dc, dm, n);
    WV_HIP(hipGetLastError());
}

void launch_absmax_fields(const float* states, long long nstates, long long N, double* d_out4,
                          hipStream_t st)
{
    const int nb = 1024;
    double* partial = nullptr;
    WV_HIP(hipMallocAsync((void**)&partial, sizeof(double) * 4 * nb, st));
    hipLaunchKernelGGL(absmax_kernel, dim3(nb, 4), dim3(RB), 0, st, states, nstates, N, partial);
    hipLaunchKernelGGL(absmax_finalize, dim3(1), dim3(64), 0, st, partial, nb, d_out4);
    WV_HIP(hipGetLastError());
    WV_HIP(hipFreeAsync(partial, st));
}

}  // namespace wv
