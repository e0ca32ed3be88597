// Exact storage of the largest-range patches alongside the autoencoder latents
// (error bounding): per compressed state, select the K patches with the largest
// e-field range r (ties: lower patch index first), keep their e values, and
// restore them after decompression.

#include "ae_internal.h"

namespace wv {
namespace {

constexpr int SEL_THREADS = 1024;

// inclusive block scan of one int per thread
__device__ int block_scan_incl(int v, int* sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int o = 1; o < SEL_THREADS; o <<= 1) {
        const int t = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    const int r = sh[tid];
    __syncthreads();
    return r;
}

// keys: r_e = meta[p*8 + 1] > 0, ordered as uint32 bit patterns. Radix select
// (8 bits per pass, most significant first) finds the K-th largest key T; the
// output lists, in increasing patch order, every patch with key > T and the
// first (K - #{key > T}) patches with key == T.
__global__ void __launch_bounds__(SEL_THREADS) topk_kernel(const float* __restrict__ meta, int P, int K,
                                                          int* __restrict__ out)
{
    __shared__ unsigned hist[256];
    __shared__ unsigned s_prefix, s_mask;
    __shared__ int s_rem;
    __shared__ int sh[SEL_THREADS];
    const int tid = threadIdx.x;
    unsigned prefix = 0, mask = 0;
    int rem = K;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int b = tid; b < 256; b += SEL_THREADS) hist[b] = 0;
        __syncthreads();
        for (int p = tid; p < P; p += SEL_THREADS) {
            const unsigned key = __float_as_uint(meta[(long long)p * 8 + 1]);
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            int cum = 0, d = 255;
            for (; d > 0; --d) {
                if (cum + (int)hist[d] >= rem) break;
                cum += (int)hist[d];
            }
            s_prefix = prefix | ((unsigned)d << shift);
            s_mask = mask | (255u << shift);
            s_rem = rem - cum;
        }
        __syncthreads();
        prefix = s_prefix;
        mask = s_mask;
        rem = s_rem;
        __syncthreads();
    }
    const unsigned T = prefix;
    const int per = (P + SEL_THREADS - 1) / SEL_THREADS;
    const int p0 = min(P, tid * per), p1 = min(P, p0 + per);
    int gt = 0, eq = 0;
    for (int p = p0; p < p1; ++p) {
        const unsigned key = __float_as_uint(meta[(long long)p * 8 + 1]);
        gt += key > T;
        eq += key == T;
    }
    const int eq_before = block_scan_incl(eq, sh) - eq;
    const int take_eq = max(0, min(eq, rem - eq_before));
    const int sel = gt + take_eq;
    int pos = block_scan_incl(sel, sh) - sel;
    int eq_seen = 0;
    for (int p = p0; p < p1; ++p) {
        const unsigned key = __float_as_uint(meta[(long long)p * 8 + 1]);
        bool pick = key > T;
        if (key == T) {
            pick = eq_seen < take_eq;
            ++eq_seen;
        }
        if (pick) out[pos++] = p;
    }
}

// exc[k][l] = e of patch idx[k] at local cell l (one block per patch)
__global__ void gather_kernel(const float* __restrict__ state, int ny, int nx, int Py, int Px,
                              const int* __restrict__ idx, float* __restrict__ exc)
{
    const int k = blockIdx.x, l = threadIdx.x;
    const int p = idx[k];
    const int px = p % Px, py = (p / Px) % Py, pz = p / (Px * Py);
    const long long z = pz * 8 + (l >> 6), y = py * 8 + ((l >> 3) & 7), x = px * 8 + (l & 7);
    exc[(long long)k * 512 + l] = state[(z * ny + y) * nx + x];
}

__global__ void scatter_kernel(float* __restrict__ e, int ny, int nx, int Py, int Px, const int* __restrict__ idx,
                               const float* __restrict__ exc)
{
    const int k = blockIdx.x, l = threadIdx.x;
    const int p = idx[k];
    const int px = p % Px, py = (p / Px) % Py, pz = p / (Px * Py);
    const long long z = pz * 8 + (l >> 6), y = py * 8 + ((l >> 3) & 7), x = px * 8 + (l & 7);
    e[(z * ny + y) * nx + x] = exc[(long long)k * 512 + l];
}

}  // namespace

void exceptions_store(const PatchGrid& pg, const float* state, const float* meta, int K, int* idx, float* exc,
                      hipStream_t st)
{
    if (K <= 0) return;
    WV_REQUIRE(K <= pg.P, WV_EINVAL, "more exception patches than patches");
    hipLaunchKernelGGL(topk_kernel, dim3(1), dim3(SEL_THREADS), 0, st, meta, (int)pg.P, K, idx);
    hipLaunchKernelGGL(gather_kernel, dim3(K), dim3(512), 0, st, state, pg.ny, pg.nx, pg.ny / 8, pg.nx / 8, idx, exc);
    WV_HIP(hipGetLastError());
}

void exceptions_restore(const PatchGrid& pg, float* e, int K, const int* idx, const float* exc, hipStream_t st)
{
    if (K <= 0) return;
    hipLaunchKernelGGL(scatter_kernel, dim3(K), dim3(512), 0, st, e, pg.ny, pg.nx, pg.ny / 8, pg.nx / 8, idx, exc);
    WV_HIP(hipGetLastError());
}

}  // namespace wv
