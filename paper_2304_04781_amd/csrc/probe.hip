// Streaming probe: the HBM rate a plain element-wise kernel reaches with a given
// mix of input and output arrays (the stencils' mixes: 5 arrays read and 4 written
// per cell forward, about 7 and 5 adjoint). It is the practical ceiling the stencil
// kernels are compared with, next to the published peak; it plays no part in the
// solves.
//
// One thread per float4 of every array: loads of all inputs, their sum, and the
// sum scaled by (q + 1) stored to output q with non-temporal stores (the stencils'
// output policy). 256 threads per work-group, so a 64 MiB array gives 16,384
// work-groups.

#include "wv_internal.h"

namespace wv {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int NIN, int NOUT>
__global__ void __launch_bounds__(256) stream_kernel(const f32x4* __restrict__ in, f32x4* __restrict__ out,
                                                     long long n4)
{
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n4) return;
    f32x4 s = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NIN; ++q) s += __builtin_nontemporal_load(in + q * n4 + i);
#pragma unroll
    for (int q = 0; q < NOUT; ++q) __builtin_nontemporal_store(s * (float)(q + 1), out + q * n4 + i);
}

template <int NIN, int NOUT>
void launch(const float* in, float* out, long long n, hipStream_t st)
{
    const long long n4 = n / 4;
    hipLaunchKernelGGL((stream_kernel<NIN, NOUT>), dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<const f32x4*>(in), reinterpret_cast<f32x4*>(out), n4);
}

template <class F>
int guarded_probe(F&& f)
{
    try {
        return f();
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    }
}

}  // namespace
}  // namespace wv

extern "C" int wv_stream_probe(const float* in, float* out, int32_t n_in, int32_t n_out, int64_t n, int32_t reps,
                               void* stream, double* h_us)
{
    using namespace wv;
    return guarded_probe([&]() -> int {
        WV_REQUIRE(in && out && h_us && reps >= 1, WV_EINVAL, "null buffer or reps < 1");
        WV_REQUIRE(n > 0 && n % 4 == 0 && n / 4 / 256 < (1LL << 31), WV_EINVAL,
                   "n must be a positive multiple of 4 below 2^41");
        void (*fn)(const float*, float*, long long, hipStream_t) = nullptr;
        if (n_in == 1 && n_out == 1) fn = launch<1, 1>;
        if (n_in == 5 && n_out == 4) fn = launch<5, 4>;
        if (n_in == 7 && n_out == 5) fn = launch<7, 5>;
        WV_REQUIRE(fn, WV_EINVAL, "supported mixes (inputs, outputs): (1, 1), (5, 4), (7, 5)");
        const hipStream_t st = (hipStream_t)stream;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        WV_HIP(hipEventCreate(&e0));
        WV_HIP(hipEventCreate(&e1));
        fn(in, out, n, st);  // warm-up
        WV_HIP(hipGetLastError());
        WV_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) fn(in, out, n, st);
        WV_HIP(hipEventRecord(e1, st));
        WV_HIP(hipGetLastError());
        WV_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        WV_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *h_us = 1e3 * (double)ms / reps;
        return WV_OK;
    });
}
