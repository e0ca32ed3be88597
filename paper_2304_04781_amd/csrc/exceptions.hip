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
// first (K - #{key > T}) patches with key == T. Each thread keeps a contiguous
// run of up to KPT keys in registers; histograms are per wave to limit LDS
// atomic contention (many patches share the floor value beta).
constexpr int NWAVE = SEL_THREADS / 64;
constexpr int KPT_MAX = 128;  // keys per thread: up to 131072 patches

template <int KPT>
__global__ void __launch_bounds__(SEL_THREADS) topk_kernel(const float* __restrict__ meta, int P, int K,
                                                          int* __restrict__ out)
{
    __shared__ unsigned hist[NWAVE][256];
    __shared__ unsigned tot[256];
    __shared__ unsigned s_prefix, s_mask;
    __shared__ int s_rem;
    __shared__ int sh[SEL_THREADS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (P + SEL_THREADS - 1) / SEL_THREADS;
    const int p0 = min(P, tid * per), p1 = min(P, p0 + per);
    unsigned key[KPT];
#pragma unroll
    for (int q = 0; q < KPT; ++q) key[q] = (p0 + q < p1) ? __float_as_uint(meta[(long long)(p0 + q) * 8 + 1]) : 0u;
    const int nk = p1 - p0;

    unsigned prefix = 0, mask = 0;
    int rem = K;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int b = lane; b < 256; b += 64) hist[wave][b] = 0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            // one LDS atomic per distinct digit in the wave (many keys share the floor value)
            const unsigned d = (key[q] >> shift) & 255u;
            bool pending = q < nk && (key[q] & mask) == prefix;
            while (__any(pending)) {
                const unsigned long long live = __ballot(pending);
                const int leader = __ffsll((long long)live) - 1;
                const unsigned ld = __shfl(d, leader, 64);
                const unsigned long long same = __ballot(pending && d == ld);
                if (lane == leader) atomicAdd(&hist[wave][ld], (unsigned)__popcll(same));
                if (d == ld) pending = false;
            }
        }
        __syncthreads();
        if (tid < 256) {
            unsigned t = 0;
            for (int w = 0; w < NWAVE; ++w) t += hist[w][tid];
            tot[tid] = t;
        }
        __syncthreads();
        if (wave == 0) {
            // digits 255..0 as 64 lanes x 4: suffix sums from the top
            unsigned c4[4], s = 0;
            for (int t = 0; t < 4; ++t) {
                c4[t] = tot[255 - (lane * 4 + t)];
                s += c4[t];
            }
            unsigned incl = s;  // inclusive prefix over lanes (lane 0 = highest digits)
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            unsigned before = incl - s;
            int found = -1;
            unsigned cum_at = 0;
            for (int t = 0; t < 4; ++t) {
                if (found < 0 && before + c4[t] >= (unsigned)rem) {
                    found = 255 - (lane * 4 + t);
                    cum_at = before;
                }
                before += c4[t];
            }
            // the first lane (highest digits) that found the crossing wins
            const unsigned long long ball = __ballot(found >= 0);
            const int winner = ball ? __ffsll((long long)ball) - 1 : 63;
            const int d = __shfl(found, winner, 64);
            const unsigned cum = __shfl(cum_at, winner, 64);
            if (lane == 0) {
                const int dd = d < 0 ? 0 : d;
                s_prefix = prefix | ((unsigned)dd << shift);
                s_mask = mask | (255u << shift);
                s_rem = rem - (int)cum;
            }
        }
        __syncthreads();
        prefix = s_prefix;
        mask = s_mask;
        rem = s_rem;
        __syncthreads();
    }
    const unsigned T = prefix;
    int gt = 0, eq = 0;
#pragma unroll
    for (int q = 0; q < KPT; ++q)
        if (q < nk) {
            gt += key[q] > T;
            eq += key[q] == T;
        }
    const int eq_before = block_scan_incl(eq, sh) - eq;
    const int take_eq = max(0, min(eq, rem - eq_before));
    const int sel = gt + take_eq;
    int pos = block_scan_incl(sel, sh) - sel;
    int eq_seen = 0;
#pragma unroll
    for (int q = 0; q < KPT; ++q)
        if (q < nk) {
            bool pick = key[q] > T;
            if (key[q] == T) {
                pick = eq_seen < take_eq;
                ++eq_seen;
            }
            if (pick) out[pos++] = p0 + q;
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
    WV_REQUIRE(pg.P <= (long long)KPT_MAX * SEL_THREADS, WV_EINVAL, "too many patches for the exception selector");
    if (pg.P <= 16LL * SEL_THREADS)
        hipLaunchKernelGGL(topk_kernel<16>, dim3(1), dim3(SEL_THREADS), 0, st, meta, (int)pg.P, K, idx);
    else if (pg.P <= 32LL * SEL_THREADS)
        hipLaunchKernelGGL(topk_kernel<32>, dim3(1), dim3(SEL_THREADS), 0, st, meta, (int)pg.P, K, idx);
    else if (pg.P <= 64LL * SEL_THREADS)
        hipLaunchKernelGGL(topk_kernel<64>, dim3(1), dim3(SEL_THREADS), 0, st, meta, (int)pg.P, K, idx);
    else
        hipLaunchKernelGGL(topk_kernel<KPT_MAX>, dim3(1), dim3(SEL_THREADS), 0, st, meta, (int)pg.P, K, idx);
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
